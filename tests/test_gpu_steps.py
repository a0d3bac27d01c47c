"""GPU parity of each step of the path against the oracle: degree, histograms,
power-law fit, CSR, BFS, label + filter, routes R0 / heuristic / router, and
the router network kernels."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev
from oracle import degree as odeg
from oracle import hybrid, ks, mlp

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")

SMALL = ["gnm64k", "rmat16", "grid512", "plcomp1m", "rmat18noisy"]
KS_TOL = 1e-9


@pytest.fixture(scope="module", params=SMALL)
def graph(request):
    return gen.workload(request.param)


def test_degree_exact(graph):
    say(f"[gpu] degree {graph.name}")
    d = ccmi.degree(to_dev(graph.u), to_dev(graph.v), graph.n)
    assert np.array_equal(d.cpu().numpy(), odeg.degree(graph.u, graph.v, graph.n))


def test_degree_ragged_and_selfloops():
    rng = np.random.default_rng(3)
    for m in [1, 7, 255, 1000, 65537]:
        n = int(rng.integers(2, 70_000))
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        v[::5] = u[::5]
        d = ccmi.degree(to_dev(u), to_dev(v), n)
        assert np.array_equal(d.cpu().numpy(), odeg.degree(u, v, n)), m


def test_degree_range_error():
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.degree(to_dev(np.array([0, 9], np.int32)), to_dev(np.array([1, 1], np.int32)), 5)
    assert ei.value.code == ccmi.CC_ERANGE


def test_histograms_exact(graph):
    say(f"[gpu] histograms {graph.name}")
    deg = odeg.degree(graph.u, graph.v, graph.n)
    h64, hx, tail, tcount, amax = ccmi.degree_histograms(to_dev(deg))
    e64, ex, etail = odeg.histograms(deg)
    assert np.array_equal(h64.cpu().numpy(), e64)
    assert np.array_equal(hx.cpu().numpy(), ex)
    assert tcount == etail.shape[0]
    assert np.array_equal(np.sort(tail.cpu().numpy()), etail)
    assert amax == hybrid.choose_seed(deg)


def test_histograms_tail_and_ties():
    # degrees above 4096 and ties for the maximum (smallest id wins)
    deg = np.zeros(20_000, np.int32)
    deg[[5, 17, 9000]] = 7000
    deg[100:5000] = np.arange(4900) % 5000
    h64, hx, tail, tcount, amax = ccmi.degree_histograms(to_dev(deg))
    e64, ex, etail = odeg.histograms(deg)
    assert np.array_equal(h64.cpu().numpy(), e64) and np.array_equal(hx.cpu().numpy(), ex)
    assert np.array_equal(np.sort(tail.cpu().numpy()), etail) and amax == 5


def _ks_compare(vals_hist, tail):
    got = ccmi.powerlaw_ks(vals_hist, tail)
    v, c = odeg.distribution_from_histograms(np.asarray(vals_hist), np.asarray(tail))
    exp = ks.fit(v, c)
    say(f"   ks gpu={got['ks']:.12g} oracle={exp['ks']:.12g} alpha {got['alpha']:.10g}/{exp['alpha']:.10g} "
        f"dmin {got['dmin']}/{exp['dmin']}")
    if math.isinf(exp["ks"]):
        assert math.isinf(got["ks"])
        return got
    assert abs(got["ks"] - exp["ks"]) <= KS_TOL
    assert got["candidates"] == exp["candidates"]
    if got["dmin"] == exp["dmin"]:
        assert abs(got["alpha"] - exp["alpha"]) <= 1e-8 * exp["alpha"]
        assert got["ntail"] == exp["ntail"]
    return got


def test_powerlaw_fit_vs_oracle(graph):
    deg = odeg.degree(graph.u, graph.v, graph.n)
    _, ex, etail = odeg.histograms(deg)
    _ks_compare(ex, etail.astype(np.int32))


def test_powerlaw_fit_exact_law_and_edge_cases():
    d = np.arange(1, 3000)
    pmf = d.astype(float) ** -2.9
    cnt = np.round(1e12 * pmf / pmf.sum()).astype(np.int64)
    hx = np.zeros(4096, np.int64)
    hx[d] = cnt
    got = _ks_compare(hx, np.zeros(0, np.int32))
    assert abs(got["alpha"] - 2.9) < 1e-2
    # no candidate cutoff -> +inf
    hx = np.zeros(4096, np.int64)
    hx[3] = 10
    assert math.isinf(ccmi.powerlaw_ks(hx, np.zeros(0, np.int32))["ks"])


def test_powerlaw_fit_interior_cutoff_many_candidates():
    """More than 256 candidate cutoffs, so a strided sample is fitted in full
    first and the other candidates stop once they cannot be the best; the best
    cutoff lies inside the range (a bell-shaped body, then a noisy power-law
    tail), and degrees above 4096 go through the tail list."""
    rng = np.random.default_rng(1607)
    d = np.arange(1, 6000)
    body = np.exp(-0.5 * ((np.log(d) - np.log(12.0)) / 0.5) ** 2)
    tail = (d / 40.0) ** -2.3 * (d >= 40)
    pmf = (body + 0.6 * tail) * rng.lognormal(0.0, 0.05, d.size)
    cnt = np.round(2e9 * pmf / pmf.sum()).astype(np.int64)
    hx = np.zeros(4096, np.int64)
    hx[d[d < 4096]] = cnt[d < 4096]
    big = d[d >= 4096]
    tail_list = np.repeat(big, cnt[d >= 4096]).astype(np.int32)
    got = _ks_compare(hx, rng.permutation(tail_list))
    assert got["candidates"] > 256
    assert 10 < got["dmin"] < 4000


def test_csr_exact(graph):
    say(f"[gpu] csr {graph.name}")
    off, adj, deg = ccmi.csr(to_dev(graph.u), to_dev(graph.v), graph.n)
    eoff, eadj = hybrid.csr(graph.u, graph.v, graph.n)
    off = off.cpu().numpy()
    assert np.array_equal(off, eoff)
    assert np.array_equal(deg.cpu().numpy(), np.diff(eoff))
    # each row holds the same multiset of neighbours
    rows = np.repeat(np.arange(graph.n), np.diff(eoff))
    got = np.lexsort((adj.cpu().numpy(), rows))
    exp = np.lexsort((eadj, rows))
    assert np.array_equal(adj.cpu().numpy()[got], eadj[exp])


def test_bfs_visited_exact(graph):
    off, adj, deg = ccmi.csr(to_dev(graph.u), to_dev(graph.v), graph.n)
    d = deg.cpu().numpy()
    seeds = [hybrid.choose_seed(d), int(np.random.default_rng(1).integers(0, graph.n))]
    for s in seeds:
        say(f"[gpu] bfs {graph.name} seed={s}")
        vis, levels, bu = ccmi.bfs(off, adj, graph.n, s)
        bits = np.unpackbits(vis.cpu().numpy().view(np.uint8), bitorder="little")[: graph.n].astype(bool)
        exp = hybrid.bfs_visited(graph.u, graph.v, graph.n, s)
        assert np.array_equal(bits, exp)
        assert levels == hybrid.bfs_levels(graph.u, graph.v, graph.n, s)


def test_bfs_filter_exact(graph):
    u, v = to_dev(graph.u), to_dev(graph.v)
    off, adj, deg = ccmi.csr(u, v, graph.n)
    r = hybrid.bfs_route(graph.u, graph.v, graph.n)
    vis, _, _ = ccmi.bfs(off, adj, graph.n, r["seed"])
    labels, fu, fv, label = ccmi.bfs_filter(u, v, graph.n, vis)
    assert label == r["label"]
    exp_lab = np.where(r["visited"], r["label"], np.arange(graph.n))
    assert np.array_equal(labels.cpu().numpy(), exp_lab)
    got = np.sort(fu.cpu().numpy().astype(np.int64) * graph.n + fv.cpu().numpy())
    exp = np.sort(r["u"].astype(np.int64) * graph.n + r["v"])
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("route", ["bfs+sv", "heuristic", "auto"])
def test_routes_exact(graph, route):
    lab, st = ccmi.label(to_dev(graph.u), to_dev(graph.v), graph.n, route=route, stats=True)
    say(f"[gpu] {graph.name} {route}: took {st['route_name']} ks={st['ks_statistic']:.4g} "
        f"bfs_levels={st['bfs_levels']} visited={st['bfs_visited']} after_filter={st['edges_after_filter']} "
        f"passes={st['sv_passes']}")
    assert_labels_equal(lab, oracle_labels(graph), f"{graph.name}/{route}")
    if route in ("heuristic", "auto") and not ccmi.router_loaded():
        deg = odeg.degree(graph.u, graph.v, graph.n)
        v, c = odeg.distribution(deg)
        exp = ks.fit(v, c)
        assert abs(st["ks_statistic"] - exp["ks"]) <= KS_TOL
        assert st["route"] == (ccmi.R0_BFS_SV if ks.decide_bfs(exp["ks"]) else ccmi.R1_SV)
    if st["route"] == ccmi.R0_BFS_SV:
        r = hybrid.bfs_route(graph.u, graph.v, graph.n)
        assert st["bfs_seed"] == r["seed"] and st["bfs_label"] == r["label"]
        assert st["bfs_visited"] == int(r["visited"].sum())
        assert st["edges_after_filter"] == r["u"].shape[0]


def _star_and_lattice(leaves, side, rng):
    """A star (the largest degree) beside a side x side lattice with self-loops
    and repeated edges; ids shuffled."""
    n = 1 + leaves + side * side
    u = [np.zeros(leaves, np.int64)]
    v = [np.arange(1, leaves + 1)]
    g = 1 + leaves + np.arange(side * side).reshape(side, side)
    u += [g[:, :-1].ravel(), g[:-1, :].ravel()]
    v += [g[:, 1:].ravel(), g[1:, :].ravel()]
    loops = rng.choice(g.ravel(), 300, replace=False)
    u.append(loops)
    v.append(loops)
    u = np.concatenate(u)
    v = np.concatenate(v)
    rep = rng.choice(u.shape[0], 500, replace=False)
    u = np.concatenate([u, v[rep]])
    v = np.concatenate([v, u[rep]])
    perm = rng.permutation(n)
    return perm[u].astype(np.int32), perm[v].astype(np.int32), n


@pytest.mark.parametrize("leaves,side", [(2000, 300), (200000, 60)])
def test_bfs_route_rest_from_list_and_from_csr(leaves, side):
    """The BFS starts at the star's hub.  With the lattice holding most edges,
    the rows of the unvisited vertices hold more entries than the list has
    edges and the rest is taken from the edge list; with a big star and a
    small lattice it is read from the CSR rows (self-loops once, repeated
    edges as often as given).  Labels, the filtered count and the BFS against
    the oracle."""
    rng = np.random.default_rng(leaves + side)
    u, v, n = _star_and_lattice(leaves, side, rng)
    say(f"[gpu] bfs route rest: star {leaves} + lattice {side}^2, n={n} m={u.shape[0]}")
    lab, st = ccmi.label(to_dev(u), to_dev(v), n, route="bfs+sv", stats=True, profile=True)
    assert_labels_equal(lab, oracle.labels_uf(u, v, n), f"star{leaves}+lattice{side}")
    r = hybrid.bfs_route(u, v, n)
    assert st["bfs_seed"] == r["seed"] and st["bfs_visited"] == leaves + 1
    assert st["edges_after_filter"] == r["u"].shape[0]
    # which path read the rest: the rows of the unvisited vertices hold
    # 4 side (side - 1) entries against m edges; from the CSR rows it takes a
    # count and an emit launch, from the edge list one filter launch
    from_csr = 4 * side * (side - 1) <= u.shape[0]
    assert st["kernel_launches"][ccmi.KERNEL_CLASSES.index("filter")] == (2 if from_csr else 1)


def test_two_level_buckets_large_n():
    """n > 2^26, i.e. more than 2048 vertex buckets: the degree pass scatters
    through super-buckets first.  Degrees, the CSR and the routes that build
    it (directly, or by scattering again after the prediction) against the
    oracle; a hub sits in the last, partial super-bucket."""
    rng = np.random.default_rng(21)
    n = 70_000_003
    m = 3_000_000
    u = rng.integers(0, n, m).astype(np.int32)
    v = rng.integers(0, n, m).astype(np.int32)
    v[::7] = u[::7]
    u[:20_000] = n - 5
    g = gen.Graph(u, v, n, "large-n")
    du, dv = to_dev(u), to_dev(v)
    say("[gpu] degree large-n")
    d = ccmi.degree(du, dv, n)
    assert np.array_equal(d.cpu().numpy(), odeg.degree(u, v, n))
    say("[gpu] csr large-n")
    off, adj, deg = ccmi.csr(du, dv, n)
    eoff, eadj = hybrid.csr(u, v, n)
    assert np.array_equal(off.cpu().numpy(), eoff)
    rows = np.repeat(np.arange(n), np.diff(eoff))
    a = adj.cpu().numpy()
    assert np.array_equal(a[np.lexsort((a, rows))], eadj[np.lexsort((eadj, rows))])
    del off, adj, deg
    expect = oracle_labels(g)
    for route, kw, want in [("bfs+sv", {}, ccmi.R0_BFS_SV), ("heuristic", {"tau": 1e300}, ccmi.R0_BFS_SV),
                            ("heuristic", {"tau": 1e-300}, ccmi.R1_SV)]:
        say(f"[gpu] large-n {route} {kw}")
        lab, st = ccmi.label(du, dv, n, route=route, stats=True, **kw)
        assert st["route"] == want
        assert_labels_equal(lab, expect, f"large-n/{route}/{kw}")


def test_shipped_router_weights():
    """The trained weights shipped with the package load, pick a route on every
    workload family, and the labels stay exact (the route changes only time)."""
    import os
    path = os.path.join(os.path.dirname(ccmi.__file__), "router_weights.txt")
    ccmi.router_load(path)
    try:
        assert ccmi.router_loaded()
        for name in SMALL:
            g = gen.workload(name)
            for route in ("router", "auto"):
                lab, st = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route=route, stats=True)
                say(f"[gpu] {name} {route}: took {st['route_name']} logits={st['router_logits']}")
                assert st["route"] == int(np.argmax(st["router_logits"]))
                assert_labels_equal(lab, oracle_labels(g), f"{name}/{route}")
    finally:
        ccmi.router_set(None)
    assert not ccmi.router_loaded()


def test_route_edge_cases():
    for u, v, n in [([], [], 5), ([2], [2], 3), ([0], [1], 2), ([3, 1], [1, 3], 4)]:
        u = np.array(u, np.int32)
        v = np.array(v, np.int32)
        g = gen.Graph(u, v, n, "tiny")
        for route in ["bfs+sv", "heuristic"]:
            assert_labels_equal(ccmi.label(to_dev(u), to_dev(v), n, route=route), oracle_labels(g), f"tiny/{route}")


# ---------------------------------------------------------------- router
def _params(seed):
    ps = mlp.init_params(seed, dtype=np.float64)
    flat = np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)
    assert flat.size == ccmi.ROUTER_NPARAMS
    return ps, flat


def _unflat(flat):
    out, o = [], 0
    for shp in [(64, 66), (64,), (64, 64), (64,), (3, 64), (3,)]:
        k = int(np.prod(shp))
        out.append(flat[o:o + k].reshape(shp).astype(np.float64))
        o += k
    return out


def test_mlp_forward_vs_fp64():
    ps, flat = _params(1)
    rng = np.random.default_rng(2)
    x = rng.random((257, 66)).astype(np.float32)
    got = ccmi.mlp_forward(torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    exp, _ = mlp.forward(_unflat(flat), x.astype(np.float64))
    assert np.allclose(got, exp, rtol=1e-5, atol=1e-5)


def test_mlp_sgd_step_vs_fp64():
    _, flat = _params(3)
    rng = np.random.default_rng(4)
    x = rng.random((100, 66)).astype(np.float32)
    y = rng.integers(0, 3, 100).astype(np.int32)
    P = torch.from_numpy(flat.copy()).cuda()
    loss, g = ccmi.mlp_sgd_step(P, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 0.05, want_grads=True)
    eloss, egrads = mlp.loss_and_grads(_unflat(flat), x.astype(np.float64), y)
    eg = np.concatenate([q.reshape(-1) for q in egrads])
    assert abs(loss - eloss) <= 1e-5 * max(1.0, abs(eloss))
    assert np.allclose(g.cpu().numpy(), eg, rtol=1e-4, atol=2e-6)
    assert np.allclose(P.cpu().numpy(), flat - 0.05 * eg, rtol=1e-5, atol=1e-6)


def test_router_route_matches_fp64_argmax():
    g = gen.workload("rmat16")
    _, flat = _params(5)
    ccmi.router_set(flat)
    try:
        lab, st = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route="router", stats=True)
        assert_labels_equal(lab, oracle_labels(g), "router")
        deg = odeg.degree(g.u, g.v, g.n)
        log64, _, _ = odeg.histograms(deg)
        feats = odeg.router_features(log64, g.n, g.m).astype(np.float32).astype(np.float64)
        z, _ = mlp.forward(_unflat(flat), feats[None, :])
        assert np.allclose(st["router_logits"], z[0], rtol=1e-4, atol=1e-4)
        zs = np.sort(z[0])
        if zs[-1] - zs[-2] > 1e-3:
            assert st["route"] == int(np.argmax(z[0]))
    finally:
        ccmi.router_set(None)
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route="router")
    assert ei.value.code == ccmi.CC_ENOROUTER


def test_small_frontiers_run_in_one_workgroup():
    """Top-down levels whose frontier holds at most 65 536 adjacency entries
    run in one workgroup, many levels per launch; a larger frontier hands
    off to the launch-per-level BFS and a frontier that shrinks again comes
    back.  Cases: a 50 000-vertex path from one end (50 000 levels), a
    300-square lattice from a corner, a star of 400 000 leaves from a leaf
    (the hub's row hands off), and a broom (a 1 000-vertex path, a hub with
    200 000 leaves, a second 1 000-vertex path hanging off one leaf) from the
    first path's far end, which leaves the workgroup and comes back.  Visited
    set and level count against the oracle; the level budget of the BFS route
    still applies."""
    rng = np.random.default_rng(5)
    n = 50_000
    perm = rng.permutation(n).astype(np.int32)
    path = gen.Graph(perm[:-1], perm[1:], n, "path")
    leaves = 400_000
    star = gen.Graph(np.zeros(leaves, np.int32), np.arange(1, leaves + 1, dtype=np.int32), leaves + 1, "star")
    lat = gen.grid(300, 1.0, seed=6)
    # broom ids: path a 0..999 (999 joins the hub), hub 1000, leaves
    # 1001..201000, path b 201001..202000 hanging off leaf 1001
    hub, nl, pl = 1000, 200_000, 1000
    bu_ = [np.arange(0, pl - 1), [pl - 1], np.full(nl, hub), [hub + 1], np.arange(hub + nl + 1, hub + nl + pl)]
    bv_ = [np.arange(1, pl), [hub], np.arange(hub + 1, hub + nl + 1), [hub + nl + 1],
           np.arange(hub + nl + 2, hub + nl + pl + 1)]
    nb = hub + nl + pl + 1
    bperm = rng.permutation(nb).astype(np.int32)
    broom = gen.Graph(bperm[np.concatenate(bu_).astype(np.int64)], bperm[np.concatenate(bv_).astype(np.int64)],
                      nb, "broom")
    for g, s, handoff in ((path, int(perm[0]), False), (lat, 0, False), (star, 7, True),
                          (broom, int(bperm[0]), True)):
        say(f"[gpu] small-frontier bfs {g.name} n={g.n} seed={s}")
        off, adj, _ = ccmi.csr(to_dev(g.u), to_dev(g.v), g.n)
        vis, levels, bu = ccmi.bfs(off, adj, g.n, s)
        bits = np.unpackbits(vis.cpu().numpy().view(np.uint8), bitorder="little")[: g.n].astype(bool)
        assert np.array_equal(bits, hybrid.bfs_visited(g.u, g.v, g.n, s)), g.name
        assert levels == hybrid.bfs_levels(g.u, g.v, g.n, s), g.name
        assert (bu > 0) == handoff, (g.name, bu)
    # through the BFS route: the path's BFS is abandoned at the level budget
    # and SV labels it; the star's, from the hub, finishes in 2 levels
    lab, st = ccmi.label(to_dev(path.u), to_dev(path.v), n, route="bfs+sv", stats=True)
    assert_labels_equal(lab, np.zeros(n, np.int32), "path via bfs+sv")
    assert st["route"] == ccmi.R1_SV and st["bfs_levels"] == 256
    lab, st = ccmi.label(to_dev(star.u), to_dev(star.v), star.n, route="bfs+sv", stats=True)
    assert_labels_equal(lab, np.zeros(star.n, np.int32), "star via bfs+sv")
    assert st["route"] == ccmi.R0_BFS_SV and st["bfs_levels"] == 2 and st["bfs_visited"] == star.n


def test_degree_pass_without_count_pass():
    """Degree passes of 2^20 edges or more that need no CSR skip the count
    pass: each scatter block fills runs of fixed capacity.  Exact degrees and
    histograms on a Kronecker graph; a star whose hub overflows every run
    (the pass then runs again with the counted layout); an exact count of
    ids out of range; and the BFS route after such a prediction (its CSR
    needs the counted prefixes, built then)."""
    g = gen.workload("rmat18noisy")
    say("[gpu] capped degree pass rmat18noisy")
    d = ccmi.degree(to_dev(g.u), to_dev(g.v), g.n)
    assert np.array_equal(d.cpu().numpy(), odeg.degree(g.u, g.v, g.n))
    # sparse lists over many buckets: 2^16 edges and more take the capped layout
    rng = np.random.default_rng(17)
    for n, m in ((600_000, 1 << 16), (600_000, 100_003), (3_000_000, 400_000)):
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        say(f"[gpu] capped degree pass n={n} m={m}")
        d = ccmi.degree(to_dev(u), to_dev(v), n)
        assert np.array_equal(d.cpu().numpy(), odeg.degree(u, v, n)), (n, m)
    leaves = 1 << 21
    star = gen.Graph(np.zeros(leaves, np.int32), np.arange(1, leaves + 1, dtype=np.int32), leaves + 1, "star")
    say("[gpu] capped degree pass, star (overflow)")
    d = ccmi.degree(to_dev(star.u), to_dev(star.v), star.n)
    assert np.array_equal(d.cpu().numpy(), odeg.degree(star.u, star.v, star.n))
    lab, st = ccmi.label(to_dev(star.u), to_dev(star.v), star.n, route="heuristic", stats=True)
    assert_labels_equal(lab, np.zeros(star.n, np.int32), "star heuristic")
    assert st["max_degree"] == leaves
    # three edges out of range, counted exactly by the scatter
    u, v = g.u.copy(), g.v.copy()
    u[[5, 70_000, 3_000_000]] = [g.n, -1, g.n + 7]
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.degree(to_dev(u), to_dev(v), g.n)
    assert ei.value.code == ccmi.CC_ERANGE and "3 edges" in str(ei.value)
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(to_dev(u), to_dev(v), g.n, route="heuristic")
    assert ei.value.code == ccmi.CC_ERANGE
    # the heuristic made to pick the BFS route: its CSR after a capped pass
    lab, st = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route="heuristic", tau=1e300, stats=True)
    assert st["route"] == ccmi.R0_BFS_SV
    assert_labels_equal(lab, oracle_labels(g), "rmat18noisy heuristic")


def _with_hubs(rng, n, m, hubs):
    """Uniform random edges plus, for each (hub, share), share * m more
    edges from that hub to random vertices."""
    u = [rng.integers(0, n, m)]
    v = [rng.integers(0, n, m)]
    for h, share in hubs:
        k = int(share * m)
        u.append(np.full(k, h))
        v.append(rng.integers(0, n, k))
    u, v = np.concatenate(u).astype(np.int32), np.concatenate(v).astype(np.int32)
    order = rng.permutation(u.size)
    return u[order], v[order]


def test_degree_with_hubs():
    """The degree count sends the entries of up to two hubs per bucket (found
    from a sample) to per-lane slots and folds them back: exact degrees,
    histograms and offsets with no hub, one, two and three hubs in one
    bucket (the third counts the ordinary way), hubs on a bucket's first and
    last id and a hub holding most of its bucket; through the small-list,
    the capped and the counted (CSR) layouts."""
    rng = np.random.default_rng(29)
    B = 1 << 15   # vertices per bucket
    cases = [
        # small lists (at most 4 buckets, 2^18 edges): the direct path
        (100_000, 60_000, [(0, 0.3)]),
        (100_000, 60_000, [(B - 1, 0.2), (B, 0.2), (3, 0.1), (B + 9, 0.05)]),
        # capped layout (2^16 edges and more, no CSR)
        (1 << 20, 1 << 20, []),
        (1 << 20, 1 << 20, [(5, 0.01)]),
        (1 << 20, 1 << 20, [(7 * B, 0.006), (8 * B - 1, 0.006), (7 * B + 100, 0.004)]),
        (3_000_000, 1 << 20, [(2_999_999, 0.02), (B * 40 + 1, 0.001)]),
    ]
    for n, m, hubs in cases:
        u, v = _with_hubs(rng, n, m, hubs)
        want = odeg.degree(u, v, n)
        say(f"[gpu] degree with hubs n={n} m={u.size} hubs={hubs}")
        d = ccmi.degree(to_dev(u), to_dev(v), n)
        assert np.array_equal(d.cpu().numpy(), want), (n, hubs)
        off, _, deg = ccmi.csr(to_dev(u), to_dev(v), n)
        assert np.array_equal(deg.cpu().numpy(), want), (n, hubs, "csr")
        assert np.array_equal(np.diff(off.cpu().numpy()), want), (n, hubs, "offsets")
        _, st = ccmi.label(to_dev(u), to_dev(v), n, route="heuristic", stats=True)
        assert st["max_degree"] == int(want.max())


def test_tail_staging_overflow():
    """Degrees of 4096 and more are staged per block (1024 at most) and
    reserved with one atomic per block; past that a vertex takes its own
    slot.  Every vertex in the tail (far past a block's staging), a tail list
    shorter than the tail, and a bucket of the degree pass holding 1500 tail
    vertices (its K-S statistic against the oracle's fit of the exact
    degree distribution)."""
    n = 200_000
    deg = (4096 + np.arange(n) % 5000).astype(np.int32)
    say("[gpu] tail staging: every vertex in the tail")
    h64, hx, tail, tcount, amax = ccmi.degree_histograms(to_dev(deg))
    e64, ex, etail = odeg.histograms(deg)
    assert tcount == n
    assert np.array_equal(h64.cpu().numpy(), e64) and np.array_equal(hx.cpu().numpy(), ex)
    assert np.array_equal(np.sort(tail.cpu().numpy()), etail)
    assert amax == int(np.argmax(deg))
    _, _, tail2, tcount2, _ = ccmi.degree_histograms(to_dev(deg), tail_cap=5000)
    t2 = tail2.cpu().numpy()
    assert tcount2 == n and t2.size == 5000
    # each entry a tail degree, none more often than it occurs
    vals, cnt = np.unique(t2, return_counts=True)
    ev, ec = np.unique(etail, return_counts=True)
    pos = np.searchsorted(ev, vals)
    assert np.all(ev[pos] == vals) and np.all(cnt <= ec[pos])
    # the fused degree pass: 1500 vertices of bucket 0 with degree 4100
    rng = np.random.default_rng(41)
    nv = 1 << 20
    hubs = np.repeat(np.arange(1500, dtype=np.int32), 4100)
    others = rng.integers(1 << 15, nv, hubs.size).astype(np.int32)
    u = np.concatenate([hubs, rng.integers(0, nv, 1 << 20).astype(np.int32)])
    v = np.concatenate([others, rng.integers(0, nv, 1 << 20).astype(np.int32)])
    say(f"[gpu] tail staging: degree pass, m={u.size}")
    d = ccmi.degree(to_dev(u), to_dev(v), nv)
    want = odeg.degree(u, v, nv)
    assert np.array_equal(d.cpu().numpy(), want)
    _, st = ccmi.label(to_dev(u), to_dev(v), nv, route="heuristic", stats=True)
    vals, cnts = odeg.distribution(want)
    exp = ks.fit(vals, cnts)
    assert abs(st["ks_statistic"] - exp["ks"]) <= KS_TOL, (st["ks_statistic"], exp["ks"])
    assert st["max_degree"] == int(want.max())


def test_csr_after_capped_prediction():
    """After a capped prediction the BFS route's CSR takes its per-block
    prefixes from the prediction's fill counts instead of counting the edges
    again: one chunk per scatter block (R-MAT scale 18) and two (scale 21,
    512 chunks over 256 blocks).  Labels exact against the oracle."""
    for scale in (18, 21):
        g = gen.rmat(scale, 16.0, seed=61 + scale, noise=0.1)
        say(f"[gpu] CSR after a capped prediction, R-MAT scale {scale}, m={g.m}")
        lab, st = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route="heuristic", tau=1e300, stats=True)
        assert st["route"] == ccmi.R0_BFS_SV
        assert_labels_equal(lab, oracle_labels(g), f"rmat{scale} R0 after capped prediction")
