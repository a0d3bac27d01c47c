"""GPU tests at the size limits of the ABI.  Past n = 2^29 vertices or
m = 2^31 edges the bucketed degree pass (prediction, CSR) does not apply, and
every route falls back to SV, whose edge counts are 64-bit."""
import numpy as np
import pytest
import torch

import gen
from gpu_util import oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")


def test_more_than_2_29_vertices():
    """n = 600M, 1M random edges among the first 3M ids and a few at the top:
    the heuristic and the BFS route fall back to SV (R1).  Expected labels from
    the oracle on the ids that occur (the compression keeps their order, so
    component minima map to component minima)."""
    rng = np.random.default_rng(31)
    n = 600_000_000
    u = rng.integers(0, 3_000_000, 1_000_000).astype(np.int32)
    v = rng.integers(0, 3_000_000, 1_000_000).astype(np.int32)
    u = np.concatenate([u, np.array([n - 1, n - 2, 0, 123_456_789], np.int32)])
    v = np.concatenate([v, np.array([n - 2, 123_456_789, 5, n - 1], np.int32)])
    ids, inv = np.unique(np.concatenate([u, v]), return_inverse=True)
    cu, cv = inv[: u.size].astype(np.int32), inv[u.size:].astype(np.int32)
    small = oracle_labels(gen.Graph(cu, cv, int(ids.size), "compressed"))
    du, dv = to_dev(u), to_dev(v)
    for route in ("heuristic", "bfs+sv"):
        say(f"[gpu] n = 600M, route {route}")
        lab, st = ccmi.label(du, dv, n, route=route, stats=True)
        assert st["route"] == ccmi.R1_SV
        got = lab.cpu().numpy()
        del lab
        assert np.array_equal(got[ids], ids[small])
        rest = np.ones(n, bool)
        rest[ids] = False
        assert np.array_equal(got[rest], np.flatnonzero(rest).astype(np.int32))
        del got, rest
    ccmi.release_workspace()


def test_at_least_2_31_edges():
    """m = 2^31 + 3 edges (17 GB of ids, built on the GPU): an ordered cycle
    over N = 2^21 vertices repeated 1024 times, plus an edge joining two of
    the 5 vertices past it.  Labels: 0 on the cycle, N + 3 for the pair, the
    vertex itself for the other three."""
    N = 1 << 21
    n = N + 5
    m = (1 << 31) + 3
    u = torch.empty(m, dtype=torch.int32, device="cuda")
    v = torch.empty(m, dtype=torch.int32, device="cuda")
    step = 1 << 28
    for a in range(0, m - 1, step):
        b = min(a + step, m - 1)
        i = torch.arange(a, b, dtype=torch.int64, device="cuda")
        u[a:b] = (i % N).to(torch.int32)
        v[a:b] = ((i + 1) % N).to(torch.int32)
        del i
    u[m - 1] = N + 3
    v[m - 1] = N + 4
    torch.cuda.synchronize()
    expect = torch.zeros(n, dtype=torch.int32)
    expect[N:] = torch.arange(N, n, dtype=torch.int32)
    expect[N + 4] = N + 3
    say(f"[gpu] m = 2^31 + 3 edges, n = {n}")
    lab, st = ccmi.label(u, v, n, route="heuristic", stats=True, max_passes=200)
    assert st["route"] == ccmi.R1_SV
    assert torch.equal(lab.cpu(), expect)
    say(f"   passes={st['sv_passes']} deep_rounds={st['sv_deep_rounds']} ms={st['ms_total']:.1f}")
    del u, v, lab
    torch.cuda.empty_cache()
    ccmi.release_workspace()
