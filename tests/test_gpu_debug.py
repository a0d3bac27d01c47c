"""GPU tests of the debug aids: the device-side invariant checks (every
parent link inside [0, x] after each SV pass; I1 and I2 on the result) and
the allocation-failure hook behind CC_ENOMEM."""
import math

import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")


def _limit(n):
    return 8 * math.ceil(math.log2(n + 1)) + 64


def test_checks_pass_on_exact_results():
    """With check on, every route on Kronecker, G(n,m), lattice and an
    ordered path (deep chains, flatten rounds) returns the exact labels, and
    the stats say the checks ran, within the pass limit."""
    n = 1 << 18
    ids = np.arange(n, dtype=np.int32)
    cases = [(gen.workload("rmat16"), ("sv", "sv-theta", "bfs+sv", "heuristic")),
             (gen.gnm(1 << 16, 1 << 16, seed=1), ("sv", "bfs+sv")),
             (gen.grid(300, 0.7, seed=3), ("sv", "sv-theta")),
             (gen.Graph(ids[:-1], ids[1:], n, "ordered path"), ("sv", "sv-theta"))]
    for g, routes in cases:
        expect = oracle_labels(g)
        u, v = to_dev(g.u), to_dev(g.v)
        for route in routes:
            say(f"[gpu] checked {g.name} {route}")
            lab, st = ccmi.label(u, v, g.n, route=route, stats=True, check=True)
            assert_labels_equal(lab, expect, f"checked {g.name}/{route}")
            assert st["check_flags"] == 1, (g.name, route, st["check_flags"])
            assert st["check_pass_limit"] == _limit(g.n)
            assert st["sv_passes"] <= st["check_pass_limit"]
    # unchecked calls report nothing
    _, st = ccmi.label(u, v, n, route="sv", stats=True)
    assert st["check_flags"] == 0 and st["check_pass_limit"] == 0


def test_check_environment_variable(monkeypatch):
    g = gen.workload("rmat16")
    u, v = to_dev(g.u), to_dev(g.v)
    monkeypatch.setenv("CCMI_CHECK", "1")
    say("[gpu] CCMI_CHECK=1")
    lab, st = ccmi.label(u, v, g.n, route="heuristic", stats=True)
    assert_labels_equal(lab, oracle_labels(g), "CCMI_CHECK=1")
    assert st["check_flags"] == 1
    monkeypatch.setenv("CCMI_CHECK", "0")
    _, st = ccmi.label(u, v, g.n, route="sv", stats=True)
    assert st["check_flags"] == 0


def _counts(lab, u, v, n):
    """I1 / I2 / range counts of a labelling, written out in numpy."""
    lab = np.asarray(lab, np.int64)
    inr = (u >= 0) & (u < n) & (v >= 0) & (v < n)
    split = int(np.count_nonzero(lab[u[inr]] != lab[v[inr]]))
    x = np.arange(n)
    ok = (lab >= 0) & (lab <= x)
    ok[ok] &= lab[lab[ok]] == lab[ok]
    return {"edges_split": split, "vertices_bad": int(np.count_nonzero(~ok)),
            "edges_out_of_range": int(np.count_nonzero(~inr))}


def test_check_labels_counts_violations():
    """cc_check_labels counts exactly what I1 and I2 say on exact and on
    corrupted labellings, and cannot see an over-merge (its documented limit)."""
    g = gen.workload("rmat16")
    expect = oracle_labels(g)
    u, v = to_dev(g.u), to_dev(g.v)
    say("[gpu] check_labels exact")
    assert ccmi.check_labels(u, v, g.n, to_dev(expect)) == {"edges_split": 0, "vertices_bad": 0,
                                                             "edges_out_of_range": 0}
    rng = np.random.default_rng(9)
    deg = np.bincount(np.concatenate([g.u, g.v]), minlength=g.n)
    nonmin = np.flatnonzero((expect != np.arange(g.n)) & (deg > 0))
    # a vertex split off its component: its edges break I1, I2 still holds
    lab = expect.copy()
    x = int(rng.choice(nonmin))
    lab[x] = x
    # a component's minimum relabelled upwards: it and every member break I2
    r = int(rng.choice(np.unique(expect[nonmin])))
    lab2 = expect.copy()
    lab2[r] = r + 1
    # two whole components merged under the smaller minimum: I1 and I2 hold
    roots = np.unique(expect)
    lab3 = expect.copy()
    lab3[expect == roots[-1]] = roots[0]
    for name, bad in (("split vertex", lab), ("raised minimum", lab2), ("over-merge", lab3)):
        say(f"[gpu] check_labels {name}")
        got = ccmi.check_labels(u, v, g.n, to_dev(bad))
        assert got == _counts(bad, g.u, g.v, g.n), name
    assert ccmi.check_labels(u, v, g.n, to_dev(lab))["edges_split"] > 0
    assert ccmi.check_labels(u, v, g.n, to_dev(lab2))["vertices_bad"] > 1
    assert ccmi.check_labels(u, v, g.n, to_dev(lab3)) == {"edges_split": 0, "vertices_bad": 0,
                                                          "edges_out_of_range": 0}
    # an edge out of range is counted, not followed
    uo = np.concatenate([g.u, np.array([g.n, 0], np.int32)])
    vo = np.concatenate([g.v, np.array([1, -5], np.int32)])
    got = ccmi.check_labels(to_dev(uo), to_dev(vo), g.n, to_dev(expect))
    assert got == {"edges_split": 0, "vertices_bad": 0, "edges_out_of_range": 2}


def test_allocation_failure_reports_enomem_and_recovers():
    """The nth allocation of a call fails (cached scratch after a release,
    pool scratch, the BFS route's larger set, the batched and 64-bit entry
    points): the call returns CC_ENOMEM, and the next call is exact."""
    g = gen.workload("rmat16")
    expect = oracle_labels(g)
    u, v = to_dev(g.u), to_dev(g.v)
    try:
        for scratch, route, nth in (("cached", "sv", 1), ("cached", "sv", 4), ("cached", "bfs+sv", 9),
                                    ("cached", "heuristic", 2), ("pool", "sv", 1), ("pool", "bfs+sv", 3)):
            say(f"[gpu] failing allocation {nth} of {scratch}/{route}")
            ccmi.release_workspace()
            ccmi.debug_fail_alloc(nth)
            with pytest.raises(ccmi.CCError) as ei:
                ccmi.label(u, v, g.n, route=route, scratch=scratch)
            assert ei.value.code == ccmi.CC_ENOMEM, str(ei.value)
            assert "out of memory" in str(ei.value).lower()
            ccmi.debug_fail_alloc(0)
            assert_labels_equal(ccmi.label(u, v, g.n, route=route, scratch=scratch), expect,
                                f"after failure {scratch}/{route}")
        b = gen.batch(16, 41, lg_hi=11.0)
        args = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (b.u, b.v, b.edge_off, b.vert_off)]
        want_b = np.concatenate([oracle_labels(b.graph(k)) for k in range(b.G)])
        say("[gpu] failing allocation of a batched call")
        ccmi.release_workspace()
        ccmi.debug_fail_alloc(1)
        with pytest.raises(ccmi.CCError) as ei:
            ccmi.label_batched(*args)
        assert ei.value.code == ccmi.CC_ENOMEM
        ccmi.debug_fail_alloc(0)
        assert np.array_equal(ccmi.label_batched(*args).cpu().numpy(), want_b)
        say("[gpu] failing allocation of a 64-bit call")
        u64 = torch.from_numpy(g.u.astype(np.int64) * 1000003 + 7).cuda()
        v64 = torch.from_numpy(g.v.astype(np.int64) * 1000003 + 7).cuda()
        ccmi.release_workspace()
        ccmi.debug_fail_alloc(2)
        with pytest.raises(ccmi.CCError) as ei:
            ccmi.label64(u64, v64)
        assert ei.value.code == ccmi.CC_ENOMEM
        ccmi.debug_fail_alloc(0)
        ids, labs = ccmi.label64(u64, v64)
        ids, labs = ids.cpu().numpy(), labs.cpu().numpy()
        # ids are x * 1000003 + 7 for the vertices in some edge
        x = (ids - 7) // 1000003
        assert np.array_equal(labs, expect[x].astype(np.int64) * 1000003 + 7)
    finally:
        ccmi.debug_fail_alloc(0)


_FAIL_CHILD = """
import sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import gen, oracle, paper_1607_06156_amd as ccmi
g = gen.workload("rmat16")
u, v = torch.from_numpy(g.u).cuda(), torch.from_numpy(g.v).cuda()
try:
    ccmi.label(u, v, g.n, route="sv")
    print("no failure")
except ccmi.CCError as e:
    print("failed", e.code)
lab = ccmi.label(u, v, g.n, route="sv").cpu().numpy()
print("exact", bool(np.array_equal(lab, oracle.labels_uf(g.u, g.v, g.n))))
"""


def test_failure_hooks_from_the_environment(monkeypatch):
    """CCMI_FAIL_ALLOC=1 (read once, at the first allocation) makes a fresh
    process's first call fail with CC_ENOMEM and its second succeed;
    CCMI_MAX_PASSES=1 (read per call) caps the passes of calls that set no
    cap, so a graph that needs more fails with CC_EINTERNAL."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CCMI_FAIL_ALLOC="1")
    say("[gpu] child with CCMI_FAIL_ALLOC=1")
    r = subprocess.run([sys.executable, "-c", _FAIL_CHILD.format(root=root)], capture_output=True, text=True,
                       env=env, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert f"failed {ccmi.CC_ENOMEM}" in r.stdout and "exact True" in r.stdout, r.stdout
    # a permuted path needs several passes
    n = 100_000
    pi = gen.permutation(n, seed=5)
    u, v = to_dev(pi[:-1]), to_dev(pi[1:])
    monkeypatch.setenv("CCMI_MAX_PASSES", "1")
    say("[gpu] CCMI_MAX_PASSES=1")
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(u, v, n, route="sv")
    assert ei.value.code == ccmi.CC_EINTERNAL
    monkeypatch.delenv("CCMI_MAX_PASSES")
    assert torch.all(ccmi.label(u, v, n, route="sv") == 0)
