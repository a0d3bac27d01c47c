"""Benchmark: connected-component labelling throughput on one MI355X.

One step = one cc_label call (the whole path: degree pass, histograms and route
decision, then BFS + filter and/or the SV passes) over the synthetic
workload, inputs already resident in HBM.  Prints one JSON line on stdout;
progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--config rmat24] [--route heuristic|router|sv|...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "CC edges/s + achieved HBM GB/s; routed/batched vs plain SV, exact labels"
WORKLOAD_DESC = {
    "rmat24": "R-MAT scale 24, edge factor 16 (a,b,c,d = .57,.19,.19,.05), ids permuted, duplicates and "
              "self-loops kept, seed 2",
    "rmat24noisy": "R-MAT scale 24, edge factor 16, per-level noise 0.1 (noisy SKG), ids permuted, seed 2",
    "gnm64k": "G(n,m) n=65536 m=65536, no self-loops or duplicates, seed 1",
    "grid8192": "8192x8192 lattice, each edge kept with p=0.7, ids permuted, edges shuffled, seed 3",
    "plcomp200m": "200M-vertex forest of power-law sized components (exponent 2.5, sizes 1..1e5), paths with "
                  "branches and chords, max degree 8, ids permuted, seed 4",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_route(ccmi, torch, u, v, n, route, steps, warmup, profile=False, **kw):
    out = torch.empty(n, dtype=torch.int32, device=u.device)
    for _ in range(warmup):
        ccmi.label(u, v, n, route=route, out=out, **kw)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = ccmi.label(u, v, n, route=route, out=out, stats=True, profile=profile, **kw)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return out, (t1 - t0) / steps, stats


def measured_traffic(cls, config):
    """HBM bytes per launch of kernel class `cls` on `config` from the committed
    rocprofv3 counter summary, or None if there is none or the kernel's source
    changed since it was taken."""
    from paper_1607_06156_amd import rocprof_summary as rs
    path = os.path.join(ROOT, "profiles", f"pmc_{cls}_{config}.txt")
    if cls not in rs.KERNEL_SOURCES or not os.path.exists(path):
        return None
    d = rs.read_pmc_file(path)
    if d.get("source_sha256") != rs.source_sha256(cls):
        log(f"[bench] {path}: kernel sources changed since the counters were taken; traffic unknown")
        return None
    return float(d["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="rmat24")
    ap.add_argument("--route", default="heuristic")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-compare", action="store_true", help="skip the forced-route comparison")
    ap.add_argument("--router-weights", default=os.path.join(ROOT, "paper_1607_06156_amd", "router_weights.txt"),
                    help="weights loaded for --route router / auto")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (batch4096 vs per-graph launches) and router-vs-heuristic legs")
    ap.add_argument("--router-graphs", type=int, default=200,
                    help="held-out graphs of the router-vs-heuristic leg")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured ceilings (cc_measure_peaks: copy, random gathers, atomicMin)")
    ap.add_argument("--tuples", default="",
                    help="comma-separated workloads: time Algorithm 1 with radix sorts (cc_label_tuples) against "
                         "the atomic-hooking SV route, one JSON line each, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(labelling is a single-device job here); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1607_06156_amd as ccmi

    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.tuples:
        for name in args.tuples.split(","):
            print(json.dumps(bench_tuples(name)), flush=True)
        return
    if args.config.startswith("batch"):
        print(json.dumps(bench_batched(args, args.config, args.steps, args.warmup)), flush=True)
        return
    if args.route in ("router", "auto"):
        ccmi.router_load(args.router_weights)

    t = time.time()
    g = gen.workload(args.config)
    log(f"[bench] generated {args.config}: n={g.n} m={g.m} in {time.time() - t:.1f}s")
    u = torch.from_numpy(g.u).cuda()
    v = torch.from_numpy(g.v).cuda()
    torch.cuda.synchronize()

    # timed region: K whole-path calls, per-kernel HIP events recorded by the library
    labels, sec, stats = time_route(ccmi, torch, u, v, g.n, args.route, args.steps, args.warmup, profile=True)
    ms = sec * 1e3
    value = g.m / sec
    st = stats[-1]
    log(f"[bench] route={st['route_name']} {ms:.3f} ms/step  {value / 1e9:.2f} G edges/s  "
        f"passes={st['sv_passes']} ks={st['ks_statistic']}")

    # dominant kernel (largest summed device time over the timed steps)
    kms = np.sum([s["kernel_ms"] for s in stats], axis=0)
    kb = np.sum([s["kernel_bytes"] for s in stats], axis=0)
    kl = np.sum([s["kernel_launches"] for s in stats], axis=0)
    dom = int(np.argmax(kms))
    achieved = (kb[dom] / (kms[dom] / 1e3)) / 1e9 if kms[dom] > 0 else 0.0
    roofline = {
        "bound": "hbm", "kernel": ccmi.KERNEL_CLASSES[dom], "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(ccmi.KERNEL_CLASSES[dom], args.config),
        "avg_launch_ms": round(float(kms[dom] / max(kl[dom], 1)), 4),
        "bytes_per_launch": float(kb[dom] / max(kl[dom], 1)),
    }
    kernels = {ccmi.KERNEL_CLASSES[i]: {"ms_per_step": round(float(kms[i]) / len(stats), 4),
                                         "launches_per_step": float(kl[i]) / len(stats),
                                         "GBps": round(float(kb[i] / (kms[i] / 1e3) / 1e9), 2) if kms[i] else None}
               for i in range(len(ccmi.KERNEL_CLASSES)) if kl[i]}
    whole_gbs = st["algorithmic_bytes"] / sec / 1e9

    extra = {}
    if not args.no_compare:
        for r in ["sv", "sv-theta", "bfs+sv"]:
            try:
                _, s2, sts = time_route(ccmi, torch, u, v, g.n, r, max(2, args.steps // 2), 1)
                extra[r] = {"ms_per_step": round(s2 * 1e3, 3), "edges_per_s": g.m / s2,
                            "passes": sts[-1]["sv_passes"]}
                log(f"[bench] forced {r}: {s2 * 1e3:.3f} ms  {g.m / s2 / 1e9:.2f} G edges/s")
            except Exception as ex:  # route not available
                extra[r] = {"error": str(ex)}
        # the same forced SV route with the other two scratch sources
        ws = torch.empty(ccmi.workspace_size(g.m, g.n, "sv"), dtype=torch.uint8, device="cuda")
        for key, kw in (("sv/scratch=pool", {"scratch": "pool"}), ("sv/caller workspace", {"workspace": ws})):
            _, s2, sts = time_route(ccmi, torch, u, v, g.n, "sv", max(2, args.steps // 2), 1, **kw)
            extra[key] = {"ms_per_step": round(s2 * 1e3, 3), "edges_per_s": g.m / s2}
            log(f"[bench] forced sv, {key}: {s2 * 1e3:.3f} ms")
        del ws

    cpu = None
    exact = None
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        expect = oracle.labels_uf(g.u, g.v, g.n)
        dt = time.perf_counter() - t0
        exact = bool(np.array_equal(labels.cpu().numpy(), expect))
        cpu = {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"full workload ({g.m} edges), sequential union-find, one thread, {dt:.2f} s",
               "host_nproc": os.cpu_count(), "host_cpu": host_cpu()}
        log(f"[bench] oracle {dt:.2f}s  {g.m / dt / 1e6:.1f} M edges/s; labels exact: {exact}")

    rec = {
        "metric": METRIC,
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOAD_DESC.get(args.config, args.config)}", "n": g.n, "m": g.m,
                   "route_requested": args.route, "route_taken": st["route_name"],
                   "router_weights": os.path.relpath(args.router_weights, ROOT) if ccmi.router_loaded() else None},
        "labels_exact_vs_oracle": exact,
        "algorithmic_GBps_whole_call": round(whole_gbs, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "stats": {k: st[k] for k in ["sv_passes", "sv_deep_rounds", "active_edges", "ks_statistic", "ks_alpha",
                                      "ks_dmin", "bfs_levels", "bfs_visited", "edges_after_filter", "ms_predict",
                                      "ms_csr", "ms_bfs", "ms_filter", "ms_sv", "ms_total"]},
        "forced_routes": extra,
    }
    if not args.no_peaks:
        # measured ceilings, outside the timed region, and the SV passes'
        # random-access rates against them: parent[] is 4n bytes (64 MiB at
        # scale 24, Infinity-Cache sized), every hook attempt is a returning
        # atomicMin on it
        pk = ccmi.measure_peaks()
        sv_ms = float(np.sum([s["kernel_ms"][0] for s in stats])) / len(stats)
        nat = float(np.mean([s["sv_atomics"] for s in stats]))
        key = "mall_64MiB" if 4 * g.n > (2 << 20) and 4 * g.n <= (256 << 20) else \
            ("l2_2MiB" if 4 * g.n <= (2 << 20) else "hbm_4GiB")
        rec["measured_ceilings"] = pk
        rec["sv_atomics"] = {"per_step": int(nat), "sv_pass_ms_per_step": round(sv_ms, 4),
                             "Gps_over_sv_pass_time": round(nat / (sv_ms * 1e-3) / 1e9, 3) if sv_ms else None,
                             "ceiling_table": key, "ceiling_Gps": pk["atomicmin_Gps"][key]}
        log(f"[bench] ceilings: copy {pk['copy_GBps']} GB/s, gathers {pk['gather_Gps']} G/s, "
            f"atomicMin {pk['atomicmin_Gps']} G/s")
    if not args.no_extras:
        # the other targets, outside the timed region: batched mode against
        # per-graph launches on the 4096-graph batch (every graph checked
        # against the oracle), and the router against the degree heuristic
        del u, v, labels
        torch.cuda.empty_cache()
        b = bench_batched(args, "batch4096", 3, 1)
        rec["batched_batch4096"] = {k: b[k] for k in ("ms_per_step", "value", "labels_exact_vs_oracle",
                                                       "per_graph_loop", "passes", "max_link")}
        rec["batched_batch4096"]["blocks"] = b["config"]["blocks"]
        rec["router_vs_heuristic"] = router_leg(args)
    print(json.dumps(rec), flush=True)


def bench_tuples(name):
    """Algorithm 1 as the paper runs it (tuple array, four radix sorts per
    iteration) against the atomic-hooking SV route on one workload: time,
    iterations and the share of the time spent sorting (Section V,
    Performance Anatomy).  Labels of the two are compared element by element."""
    import numpy as np
    import torch

    import gen
    import paper_1607_06156_amd as ccmi
    g = gen.workload(name)
    u = torch.from_numpy(g.u).cuda()
    v = torch.from_numpy(g.v).cuda()
    lab_t, st = ccmi.label_tuples(u, v, g.n)              # first call also sizes the workspace
    torch.cuda.synchronize()
    lab_t, st = ccmi.label_tuples(u, v, g.n, out=lab_t)
    lab_x, stx = ccmi.label_tuples(u, v, g.n, exclude=True)   # completed partitions set aside
    exact_x = bool(torch.equal(lab_t, lab_x))
    del lab_x
    _, sv_sec, sts = time_route(ccmi, torch, u, v, g.n, "sv", 3, 1, profile=True)
    lab_s = ccmi.label(u, v, g.n, route="sv")
    exact = bool(torch.equal(lab_t, lab_s))
    sv_sort_free = sts[-1]
    rec = {"workload": f"{name}: {WORKLOAD_DESC.get(name, name)}", "n": g.n, "m": g.m,
           "tuples": st["tuples"], "iterations": st["iterations"], "sorts": st["sorts"],
           "passes_per_sort": st["passes_per_sort"], "tuples_ms": round(st["ms_total"], 3),
           "tuples_sort_ms": round(st["ms_sort"], 3), "sort_share": round(st["ms_sort"] / st["ms_total"], 4),
           "exclusion": {"iterations": stx["iterations"], "tuples_ms": round(stx["ms_total"], 3),
                         "tuples_sort_ms": round(stx["ms_sort"], 3),
                         "sort_share": round(stx["ms_sort"] / stx["ms_total"], 4), "labels_identical": exact_x},
           "sv_ms": round(sv_sec * 1e3, 3), "sv_passes": sv_sort_free["sv_passes"],
           "sv_kernel_ms": {ccmi.KERNEL_CLASSES[i]: round(float(x), 3)
                            for i, x in enumerate(sv_sort_free["kernel_ms"]) if x},
           "labels_identical": exact}
    log(f"[bench] tuples {name}: {st['ms_total']:.1f} ms ({st['iterations']} iterations, sorts "
        f"{100 * st['ms_sort'] / st['ms_total']:.1f} %) against SV {sv_sec * 1e3:.2f} ms; identical={exact}")
    del u, v, lab_t, lab_s
    torch.cuda.empty_cache()
    return rec


def oracle_batch(b, workers):
    """Oracle labels of every graph of a batch, concatenated, on a thread pool
    (the oracle's C union-find releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    out = np.empty(int(b.vert_off[-1]), dtype=np.int32)

    def one(g):
        sub = b.graph(g)
        a = int(b.vert_off[g])
        out[a:a + sub.n] = oracle.labels_uf(sub.u, sub.v, sub.n)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, range(b.G)))
    return out


def router_leg(args):
    """Router against the K-S heuristic, end to end, over the first held-out
    graphs of the router's evaluation set (new seeds of the training families
    plus the power-law forest family, never seen in training)."""
    import paper_1607_06156_amd as ccmi
    from paper_1607_06156_amd import router_train as rt
    t = time.time()
    w = rt.load(args.router_weights)
    rep, _ = rt.evaluate(w, args.router_graphs, 20_000_000, 10.0, 20.0)
    ccmi.router_set(None)
    log(f"[bench] router vs heuristic over {rep['graphs']} held-out graphs: router {rep['router_s'] * 1e3:.1f} ms, "
        f"heuristic {rep['heuristic_s'] * 1e3:.1f} ms, best forced {rep['best_forced_s'] * 1e3:.1f} ms "
        f"({time.time() - t:.0f} s)")
    return {"graphs": rep["graphs"], "router_ms": round(rep["router_s"] * 1e3, 3),
            "heuristic_ms": round(rep["heuristic_s"] * 1e3, 3), "best_forced_ms": round(rep["best_forced_s"] * 1e3, 3),
            "router_no_slower": rep["router_no_slower"],
            "by_family_ms": {f: {"router": round(d["router_s"] * 1e3, 3), "heuristic": round(d["heuristic_s"] * 1e3, 3)}
                             for f, d in rep["by_family"].items()},
            "weights": os.path.relpath(args.router_weights, ROOT)}


def bench_batched(args, config, steps, warmup):
    """Batched mode: all graphs in one persistent launch, against a loop of
    per-graph cc_label calls (plain SV) over the same device arrays; every
    graph's labels checked against the oracle.  Returns the JSON record."""
    import numpy as np
    import torch

    import gen
    import paper_1607_06156_amd as ccmi

    t = time.time()
    b = gen.workload(config)
    m = int(b.edge_off[-1])
    n = int(b.vert_off[-1])
    log(f"[bench] generated {config}: G={b.G} n={n} m={m} in {time.time() - t:.1f}s")
    u = torch.from_numpy(b.u).cuda()
    v = torch.from_numpy(b.v).cuda()
    eo = torch.from_numpy(b.edge_off).cuda()
    vo = torch.from_numpy(b.vert_off).cuda()
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    for _ in range(max(warmup, 1)):   # the first call also autotunes the grid
        ccmi.label_batched(u, v, eo, vo, out=out)
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = ccmi.label_batched(u, v, eo, vo, out=out, stats=True)
        sts.append(st)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    value = m / sec
    st = sts[-1]
    log(f"[bench] batched: {sec * 1e3:.2f} ms/step {value / 1e9:.2f} G edges/s passes={st['passes']} "
        f"blocks={st['blocks']} max_link={st['max_link']} pass_ms={st['pass_ms']}")
    kernel_ms = float(np.mean([s["ms_total"] for s in sts]))
    # the persistent kernel is the only kernel: algorithmic bytes of one
    # launch from its own counts (the single-graph model): identity init
    # (4 B per vertex), per active edge read 8 B plus two 4 B gathers, 8 B per
    # atomic, 4 B per walk read, 8 B per survivor written, final labels
    # (8 B per vertex)
    kbytes = (12.0 * n + 16.0 * st["edges_read"] + 8.0 * st["atomics"] + 4.0 * st["chase_reads"]
              + 8.0 * st["survivors_written"])
    achieved = kbytes / (kernel_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": "batched_kernel", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic("batched", config),
                "avg_launch_ms": round(kernel_ms, 4), "bytes_per_launch": kbytes}
    # per-graph launches of the same SV kernels
    loop = None
    if not args.no_compare:
        out2 = torch.empty(n, dtype=torch.int32, device="cuda")
        offs_e = b.edge_off.tolist()
        offs_v = b.vert_off.tolist()

        def run_loop():
            for g in range(b.G):
                a, c = offs_e[g], offs_e[g + 1]
                x, y = offs_v[g], offs_v[g + 1]
                if y > x:
                    ccmi.label(u[a:c], v[a:c], y - x, route="sv", out=out2[x:y])
        run_loop()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_loop()
        torch.cuda.synchronize()
        lsec = time.perf_counter() - t0
        same = bool(torch.equal(out, out2))
        loop = {"ms": round(lsec * 1e3, 2), "edges_per_s": m / lsec, "speedup_batched_vs_loop": lsec / sec,
                "labels_identical": same}
        log(f"[bench] per-graph loop: {lsec * 1e3:.1f} ms  ({m / lsec / 1e9:.2f} G edges/s); batched is "
            f"{lsec / sec:.1f}x; identical={same}")
        del out2
    lab_h = out.cpu().numpy()
    del u, v, eo, vo, out
    torch.cuda.empty_cache()
    # every graph against the oracle, on a pool of the host's threads (the
    # cpu baseline: the oracle over the whole batch)
    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    expect = oracle_batch(b, workers)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(lab_h, expect))
    log(f"[bench] oracle over all {b.G} graphs on {workers} threads: {dt:.2f} s; labels exact: {exact}")
    cpu = None
    if not args.no_cpu:
        cpu = {"value": m / dt, "unit": "edges/s", "cores": workers, "kind": "oracle",
               "sample": f"all {b.G} graphs ({m} edges), union-find per graph on a pool of {workers} threads, "
                         f"{dt:.2f} s", "host_nproc": os.cpu_count(), "host_cpu": host_cpu()}
    return {
        "metric": METRIC,
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{config}: {b.G} graphs, log2 n ~ U[8,20], families G(n,m) / R-MAT / thinned "
                               f"lattice / power-law components, seeds 5e6+g", "n": n, "m": m,
                   "blocks": st["blocks"], "tile_edges": st["tile_edges"]},
        "labels_exact_vs_oracle": exact,
        "kernel_ms": round(kernel_ms, 3),
        "roofline": roofline,
        "passes": st["passes"],
        "pass_ms": st["pass_ms"],
        "max_link": st["max_link"],
        "per_graph_loop": loop,
        "cpu_baseline": cpu,
    }


def host_cpu() -> str | None:
    """The host CPU's model name, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
