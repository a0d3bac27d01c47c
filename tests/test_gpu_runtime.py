"""GPU tests of the runtime around the kernels: work on a non-default stream,
the workspace release, and the batched autotuner's cache file."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_side_stream_and_workspace_release():
    g = gen.workload("rmat16")
    u, v = to_dev(g.u), to_dev(g.v)
    expect = oracle_labels(g)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())   # the uploads above ran on the default stream
    with torch.cuda.stream(s):
        for route in ("sv", "heuristic", "bfs+sv"):
            say(f"[gpu] side stream {route}")
            lab = ccmi.label(u, v, g.n, route=route)
            assert_labels_equal(lab, expect, f"side stream/{route}")
        b = gen.batch(12, 77, lg_hi=12.0)
        lab_b = ccmi.label_batched(torch.from_numpy(b.u).cuda(), torch.from_numpy(b.v).cuda(),
                                   torch.from_numpy(b.edge_off).cuda(), torch.from_numpy(b.vert_off).cuda())
    s.synchronize()
    parts = [oracle_labels(b.graph(k)) for k in range(b.G)]
    assert np.array_equal(lab_b.cpu().numpy(), np.concatenate(parts))
    # the workspace is released and grown again on the next call
    ccmi.release_workspace()
    assert_labels_equal(ccmi.label(u, v, g.n, route="sv"), expect, "after release")


def _batch_args(b):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (b.u, b.v, b.edge_off, b.vert_off)]


def _expected(b):
    parts = [oracle_labels(b.graph(k)) for k in range(b.G)]
    return np.concatenate(parts) if parts else np.zeros(0, np.int32)


def test_autotune_cache_file(tmp_path, monkeypatch):
    """A newly tuned size class is written, with every class tuned so far, to
    the file named by CC_AUTOTUNE_CACHE; the stored shape is the one used."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("CC_AUTOTUNE_CACHE", str(path))
    b = gen.batch(150, 9191, lg_lo=6.0, lg_hi=9.0)   # G = 150: a size class no other test uses
    say("[gpu] autotune cache")
    lab, st = ccmi.label_batched(*_batch_args(b), stats=True)
    assert np.array_equal(lab.cpu().numpy(), _expected(b))
    assert st["blocks"] > 0                          # this process owns the persistent grid
    lines = [ln.split() for ln in path.read_text().splitlines() if "/G2^7" in ln]
    assert len(lines) == 1
    key, blocks, link = lines[0]
    assert "/batched/" in key
    assert (int(blocks), int(link)) == (st["blocks"], st["max_link"])


_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import torch
import gen
import oracle
import paper_1607_06156_amd as ccmi
b = gen.batch(40, 777, lg_hi=12.0)
args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (b.u, b.v, b.edge_off, b.vert_off)]
lab, st = ccmi.label_batched(*args, stats=True)
exp = np.concatenate([oracle.labels_uf(b.graph(k).u, b.graph(k).v, b.graph(k).n) for k in range(b.G)])
assert np.array_equal(lab.cpu().numpy(), exp)
print("ok blocks", st["blocks"], "passes", st["passes"], flush=True)
"""


def test_batched_from_a_second_process():
    """A second process labels a batch while this one, which has made
    cooperative launches, still holds the GPU.  The labels are exact whether
    its persistent launch runs or is refused (the device's global wave-sync
    resource is held here) and the disjoint-union fallback labels the batch."""
    b = gen.batch(8, 55, lg_hi=10.0)
    lab = ccmi.label_batched(*_batch_args(b))        # a cooperative launch in this process
    assert np.array_equal(lab.cpu().numpy(), _expected(b))
    say("[gpu] batched in a second process")
    r = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("ok")][-1]
    say(f"   child: {line} ({'fallback' if line.split()[2] == '0' else 'persistent grid'})")


def test_concurrent_calls_from_threads():
    """Four host threads, each on its own stream, call the library at once:
    three label single graphs (a different route each call), one labels a
    batch.  Two of the single-graph threads take stream-ordered scratch from
    the pool (no lock), the third and the batch the cached workspace under its
    lock.  Every result is exact and each thread's error slot stays its own."""
    import threading
    graphs = [gen.workload("rmat16"), gen.gnm(200_000, 300_000, seed=3), gen.grid(400, 0.6, seed=4)]
    expects = [oracle_labels(g) for g in graphs]
    b = gen.batch(20, 99, lg_hi=12.0)
    bexp = _expected(b)
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep, route in enumerate(("sv", "heuristic", "bfs+sv")):
                    if k == 3:
                        lab = ccmi.label_batched(*_batch_args(b))
                        exp = bexp
                    else:
                        g = graphs[k]
                        lab = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route=route,
                                         scratch="pool" if k < 2 else "cached")
                        exp = expects[k]
                    s.synchronize()
                    if not np.array_equal(lab.cpu().numpy(), exp):
                        errors.append(f"thread {k} call {rep}: labels differ")
            if ccmi.lib().cc_last_error() not in (b"", None):
                errors.append(f"thread {k}: error slot not empty")
        except Exception as e:   # noqa: BLE001 -- reported below
            errors.append(f"thread {k}: {e!r}")

    say("[gpu] 4 threads calling at once")
    ts = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ts)
    assert not errors, errors


def test_scratch_modes_exact():
    """The three scratch sources give the same exact labels on every route:
    stream-ordered pool allocations, the cached per-device workspace, and a
    caller block of exactly cc_workspace_size bytes (used twice in a row, the
    second time for a smaller graph)."""
    graphs = [gen.workload("rmat16"), gen.grid(300, 0.7, seed=8), gen.gnm(50_000, 40_000, seed=9)]
    for g in graphs:
        u, v = to_dev(g.u), to_dev(g.v)
        expect = oracle_labels(g)
        for route in ("sv", "sv-theta", "heuristic", "bfs+sv"):
            say(f"[gpu] scratch modes {g.name} {route}")
            assert_labels_equal(ccmi.label(u, v, g.n, route=route, scratch="pool"), expect,
                                f"{g.name}/{route}/pool")
            assert_labels_equal(ccmi.label(u, v, g.n, route=route), expect, f"{g.name}/{route}/cached")
            size = ccmi.workspace_size(g.m, g.n, route)
            ws = torch.empty(size, dtype=torch.uint8, device="cuda")
            assert_labels_equal(ccmi.label(u, v, g.n, route=route, workspace=ws), expect,
                                f"{g.name}/{route}/workspace")
            h = gen.gnm(g.n // 3, g.m // 4, seed=10)      # a smaller graph in the same block
            assert_labels_equal(ccmi.label(to_dev(h.u), to_dev(h.v), h.n, route=route, workspace=ws),
                                oracle_labels(h), f"{h.name}/{route}/workspace reused")
            with pytest.raises(ccmi.CCError):
                ccmi.label(u, v, g.n, route=route, workspace=ws[: size - 1])


def test_threads_with_their_own_workspaces():
    """Two host threads, each with its own stream and its own caller
    workspace, label different graphs at the same time, five times each,
    through every route; every result is exact."""
    import threading
    graphs = [gen.workload("rmat16"), gen.grid(500, 0.65, seed=21)]
    expects = [oracle_labels(g) for g in graphs]
    errors = []
    start = threading.Barrier(2)

    def work(k):
        try:
            g = graphs[k]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                u, v = to_dev(g.u), to_dev(g.v)
                ws = torch.empty(ccmi.workspace_size(g.m, g.n, "auto"), dtype=torch.uint8, device="cuda")
                s.synchronize()
                start.wait(timeout=60)
                for rep in range(5):
                    for route in ("sv", "heuristic", "bfs+sv", "sv-theta"):
                        lab = ccmi.label(u, v, g.n, route=route, workspace=ws)
                        s.synchronize()
                        if not np.array_equal(lab.cpu().numpy(), expects[k]):
                            errors.append(f"thread {k} rep {rep} {route}: labels differ")
        except Exception as e:   # noqa: BLE001 -- reported below
            errors.append(f"thread {k}: {e!r}")

    say("[gpu] 2 threads, own workspaces")
    ts = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=180)
    assert not any(t.is_alive() for t in ts)
    assert not errors, errors


def test_measured_ceilings():
    """cc_measure_peaks: every figure positive and below what the chip could
    ever do (copy under 9 TB/s), and random access slows as the table leaves
    the L2 and then the Infinity Cache."""
    say("[gpu] measured ceilings")
    pk = ccmi.measure_peaks()
    assert 100.0 < pk["copy_GBps"] < 9000.0, pk
    g, a = pk["gather_Gps"], pk["atomicmin_Gps"]
    assert all(x > 0 for x in list(g.values()) + list(a.values())), pk
    assert g["l2_2MiB"] > g["hbm_4GiB"] and a["l2_2MiB"] > a["hbm_4GiB"], pk
    assert pk["table_bytes"] == [2 << 20, 64 << 20, 4 << 30]
    # the device still labels correctly afterwards
    gr = gen.workload("rmat16")
    assert_labels_equal(ccmi.label(to_dev(gr.u), to_dev(gr.v), gr.n, route="sv"), oracle_labels(gr), "after peaks")
