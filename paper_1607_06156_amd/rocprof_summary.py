"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1607_06156_amd.rocprof_summary stats DIR [--title T] [--command C]
    python -m paper_1607_06156_amd.rocprof_summary pmc --fetch DIR --write DIR --kernel NAME
        --cls CLASS --copy-mib N [--last K] [--title T] [--command C]
    python -m paper_1607_06156_amd.rocprof_summary counters DIR [DIR ...] [--title T] [--command C]

`stats` condenses a `--kernel-trace --stats` run (its *_kernel_stats.csv) into
a table.  `pmc` takes two counter runs (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`,
each a *_counter_collection.csv) of a program that also ran one plain
device-to-device copy of N MiB, and converts the kernel's per-dispatch KiB
into bytes with the factor that makes the copy read and write exactly N MiB.
`counters` tabulates every counter of one or more `--pmc` runs per kernel:
dispatches, the sum over them and the average per dispatch.

The pmc summary carries `key: value` lines that bench.py reads back, among
them the SHA-256 of the kernel's source files: bench.py reports the traffic
only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join("paper_1607_06156_amd", "csrc")

# source files that decide the work and memory traffic of each kernel class
# (kernel body, shared device helpers, launch configuration)
KERNEL_SOURCES = {
    "sv_pass": ["sv.hip", "sv_device.hpp", "common.hpp", "hubs.hpp", "api.cpp"],
    "degree": ["degree.hip", "degree.hpp", "common.hpp", "route.cpp"],
    "bfs": ["bfs.hip", "bfs.hpp", "common.hpp", "route.cpp"],
    "filter": ["bfs.hip", "common.hpp", "route.cpp"],
    "batched": ["batched.hip", "batched.hpp", "batched_host.cpp", "sv_device.hpp", "common.hpp"],
}

# the rocclr blit kernel that a device-to-device hipMemcpyAsync runs
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_sha256(cls: str, rev: str | None = None) -> str:
    """SHA-256 over the kernel class's source files, from the working tree or,
    with rev, from that git revision (the one the profiled library was built
    from)."""
    import subprocess
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[cls]:
        if rev:
            data = subprocess.run(["git", "-C", ROOT, "show", f"{rev}:{CSRC}/{f}"], check=True,
                                  capture_output=True).stdout
        else:
            with open(os.path.join(ROOT, CSRC, f), "rb") as fh:
                data = fh.read()
        h.update(f.encode() + b"\0" + data + b"\0")
    return h.hexdigest()


def read_pmc_file(path: str) -> dict:
    """Parse a summary written by `pmc` into a dict of its key: value lines."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def _find(dirname: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not hits:
        sys.exit(f"no *{suffix} under {dirname}")
    return hits[0]


def _short(name: str, templ: bool = False) -> str:
    # demangled names carry namespaces and arguments: keep the bare kernel name
    # (with its template arguments if templ)
    base = name.split("(")[0].split("::")[-1].strip()
    return base if templ else base.split("<")[0].strip()


def stats_table(dirname: str) -> str:
    path = _find(dirname, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {_short(r['Name'], True)} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def pmc_per_dispatch(dirname: str, counter: str) -> dict:
    """kernel (short name) -> list of per-dispatch counter values (KiB), in
    dispatch order."""
    path = _find(dirname, "counter_collection.csv")
    per = defaultdict(lambda: defaultdict(float))
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[_short(r["Kernel_Name"])][int(did)] += float(r["Counter_Value"])
    return {k: [v[d] for d in sorted(v)] for k, v in per.items()}


def counters_table(dirs) -> str:
    """kernel x counter: dispatches, total and per-dispatch average."""
    rows = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    for d in dirs:
        path = _find(d, "counter_collection.csv")
        for r in csv.DictReader(open(path)):
            did = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
            rows[(_short(r["Kernel_Name"], True), r["Counter_Name"])][d][did] += float(r["Counter_Value"])
    lines = ["| kernel | counter | dispatches | total | per dispatch |", "|---|---|---|---|---|"]
    for (k, c) in sorted(rows):
        vals = [v for per in rows[(k, c)].values() for v in per.values()]
        tot = sum(vals)
        lines.append(f"| {k} | {c} | {len(vals)} | {tot:.6g} | {tot / max(len(vals), 1):.6g} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--command", default="")
    p = sub.add_parser("pmc")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--kernel", required=True, help="kernel function name, e.g. sv_pass_kernel")
    p.add_argument("--cls", required=True, choices=sorted(KERNEL_SOURCES))
    p.add_argument("--copy-mib", type=float, required=True)
    p.add_argument("--sources-rev", default=None, help="git revision the profiled library was built from")
    p.add_argument("--last", type=int, default=0, help="average only the kernel's last N dispatches")
    p.add_argument("--title", default="HBM traffic")
    p.add_argument("--command", default="")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--title", default="rocprofv3 counters")
    c.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.mode == "counters":
        print(f"# {a.title}\n")
        if a.command:
            print("Commands (from the repository root):\n")
            for cmd in a.command.split(" ;; "):
                print(f"    {cmd}")
            print()
        print(counters_table(a.dirs))
        return
    if a.mode == "stats":
        print(f"# {a.title}\n")
        if a.command:
            print(f"Command (from the repository root):\n\n    {a.command}\n")
        print(stats_table(a.dir))
        return
    fetch = pmc_per_dispatch(a.fetch, "FETCH_SIZE")
    write = pmc_per_dispatch(a.write, "WRITE_SIZE")
    copy_bytes = a.copy_mib * 1024 * 1024
    # the calibration copy is the largest copyBuffer dispatch of each run
    cf = max(fetch.get(COPY_KERNEL, [0.0]))
    cw = max(write.get(COPY_KERNEL, [0.0]))
    if cf <= 0 or cw <= 0:
        sys.exit("calibration copy not found in the counter runs")
    fscale = copy_bytes / cf
    wscale = copy_bytes / cw
    kf = fetch.get(a.kernel, [])
    kw = write.get(a.kernel, [])
    if a.last > 0:
        kf, kw = kf[-a.last:], kw[-a.last:]
    if not kf or not kw:
        sys.exit(f"kernel {a.kernel} not found in the counter runs")
    f_avg = sum(kf) / len(kf)
    w_avg = sum(kw) / len(kw)
    traffic = f_avg * fscale + w_avg * wscale
    print(f"# {a.title}\n")
    if a.command:
        print("Commands (from the repository root):\n")
        for c in a.command.split(" ;; "):
            print(f"    {c}")
        print()
    print(f"kernel: {a.kernel}")
    print(f"class: {a.cls}")
    if a.sources_rev:
        print(f"sources_rev: {a.sources_rev}")
    print(f"source_sha256: {source_sha256(a.cls, a.sources_rev)}")
    print(f"dispatches_fetch: {len(kf)}")
    print(f"dispatches_write: {len(kw)}")
    print(f"fetch_kib_per_dispatch: {f_avg:.1f}")
    print(f"write_kib_per_dispatch: {w_avg:.1f}")
    print(f"copy_mib: {a.copy_mib:g}")
    print(f"copy_fetch_kib: {cf:.1f}")
    print(f"copy_write_kib: {cw:.1f}")
    print(f"fetch_scale_bytes_per_kib: {fscale:.3f}")
    print(f"write_scale_bytes_per_kib: {wscale:.3f}")
    print(f"fetch_bytes_per_launch: {f_avg * fscale:.0f}")
    print(f"write_bytes_per_launch: {w_avg * wscale:.0f}")
    print(f"traffic_bytes_per_launch: {traffic:.0f}")


if __name__ == "__main__":
    main()
