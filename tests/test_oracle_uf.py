"""Pins for the union-find oracle: brute force, a library routine, closed forms,
invariants, the paper's worked example, and planted mistakes that must fail."""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def canonical_from_scipy(u, v, n):
    """scipy component ids -> minimum vertex id per component."""
    if n == 0:
        return np.zeros(0, np.int32)
    a = sp.coo_matrix((np.ones(len(u)), (np.asarray(u), np.asarray(v))), shape=(n, n)).tocsr()
    _, comp = connected_components(a, directed=False)
    mins = np.full(comp.max() + 1, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


def check_invariants(u, v, n, lab):
    """I1-I3 of the contract; returns a list of violated names."""
    bad = []
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    lab = np.asarray(lab, np.int64)
    if u.shape[0] and not np.array_equal(lab[u], lab[v]):
        bad.append("I1 endpoints share a label")
    x = np.arange(n)
    if np.any(lab > x):
        bad.append("I2 label <= id")
    if n and not np.array_equal(lab[lab], lab):
        bad.append("I2 label idempotent")
    return bad


# ------------------------------------------------------------ brute force
def test_all_graphs_on_five_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        u = [a for a, _ in es]
        v = [b for _, b in es]
        assert np.array_equal(oracle.labels_uf(u, v, 5), oracle.labels_bfs_brute(u, v, 5)), es


def test_all_relabelings_n4():
    """I4 permutation equivariance over every graph and every relabeling on 4 vertices."""
    pairs = list(itertools.combinations(range(4), 2))
    perms = list(itertools.permutations(range(4)))
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        u = np.array([a for a, _ in es], np.int32)
        v = np.array([b for _, b in es], np.int32)
        base = oracle.labels_uf(u, v, 4)
        for pi in perms:
            pi = np.array(pi)
            lab = oracle.labels_uf(pi[u], pi[v], 4) if len(es) else oracle.labels_uf(u, v, 4)
            # component of pi(x) in the relabelled graph = pi(component of x)
            for x in range(4):
                comp = [y for y in range(4) if base[y] == base[x]]
                assert lab[pi[x]] == min(pi[y] for y in comp)


def test_random_multigraphs_vs_brute():
    rng = np.random.default_rng(11)
    for trial in range(400):
        n = int(rng.integers(1, 13))
        m = int(rng.integers(0, 3 * n + 1))
        u = rng.integers(0, n, m)
        v = rng.integers(0, n, m)
        if m and trial % 3 == 0:
            v[: m // 3] = u[: m // 3]          # self-loops
        if m and trial % 4 == 0:
            u = np.concatenate([u, u])          # duplicates
            v = np.concatenate([v, v])
        assert np.array_equal(oracle.labels_uf(u, v, n), oracle.labels_bfs_brute(u, v, n))


@pytest.mark.parametrize("name,g", [
    ("gnm", lambda: gen.gnm(200_000, 180_000, seed=7)),
    ("rmat", lambda: gen.rmat(17, 8, seed=8)),
    ("grid", lambda: gen.grid(300, 0.55, seed=9)),
    ("plcomp", lambda: gen.plcomp(300_000, seed=10)),
])
def test_vs_scipy(name, g):
    g = g()
    lab = oracle.labels_uf(g.u, g.v, g.n)
    assert np.array_equal(lab, canonical_from_scipy(g.u, g.v, g.n))
    assert check_invariants(g.u, g.v, g.n, lab) == []


# ------------------------------------------------------------ closed forms
def test_hamiltonian_path_permuted():
    n = 50_000
    pi = gen.permutation(n, seed=3)
    assert np.all(oracle.labels_uf(pi[:-1], pi[1:], n) == 0)


def test_complete_grid_permuted():
    g = gen.grid(200, 1.0, seed=4)
    assert g.m == 2 * 200 * 199
    assert np.all(oracle.labels_uf(g.u, g.v, g.n) == 0)


def test_no_edges_identity():
    n = 1000
    e = np.zeros(0, np.int32)
    assert np.array_equal(oracle.labels_uf(e, e, n), np.arange(n))


def test_perfect_matching():
    n = 10_000
    u = np.arange(0, n, 2)
    v = u + 1
    rng = np.random.default_rng(0)
    flip = rng.random(u.shape[0]) < 0.5
    uu, vv = np.where(flip, v, u), np.where(flip, u, v)
    assert np.array_equal(oracle.labels_uf(uu, vv, n), 2 * (np.arange(n) // 2))


def test_self_loops_only_identity():
    n = 777
    x = np.arange(n)
    assert np.array_equal(oracle.labels_uf(x, x, n), x)


def test_star():
    n = 5000
    c = 1234
    leaves = np.array([x for x in range(n) if x != c])
    assert np.all(oracle.labels_uf(np.full(n - 1, c), leaves, n) == 0)
    # star on a subset: label is the smallest id among centre and leaves
    sub = np.array([4000, 4100, 4200, 4999])
    lab = oracle.labels_uf(np.full(3, 4200), np.array([4000, 4100, 4999]), n)
    assert np.all(lab[sub] == 4000)
    assert lab[17] == 17


def test_disjoint_cliques():
    n = 3000
    pi = gen.permutation(n, seed=5)
    groups = np.array_split(pi, 60)
    us, vs = [], []
    for grp in groups:
        a, b = np.triu_indices(len(grp), 1)
        us.append(grp[a])
        vs.append(grp[b])
    lab = oracle.labels_uf(np.concatenate(us), np.concatenate(vs), n)
    for grp in groups:
        assert np.all(lab[grp] == grp.min())


# ------------------------------------------------------------ invariances
def test_edge_order_orientation_duplicates_selfloops():
    g = gen.gnm(20_000, 15_000, seed=12)
    base, unions = oracle.labels_uf(g.u, g.v, g.n, return_unions=True)
    # I3: component count = n - successful unions
    assert oracle.component_count(base) == g.n - unions
    rng = np.random.default_rng(1)
    order = rng.permutation(g.m)
    swap = rng.random(g.m) < 0.5
    u2 = np.where(swap, g.v, g.u)[order]
    v2 = np.where(swap, g.u, g.v)[order]
    extra = rng.integers(0, g.m, 2000)
    loops = rng.integers(0, g.n, 500)
    u3 = np.concatenate([u2, g.u[extra], loops])
    v3 = np.concatenate([v2, g.v[extra], loops])
    assert np.array_equal(oracle.labels_uf(u3, v3, g.n), base)


def test_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.labels_uf([0, 5], [1, 2], 5)
    with pytest.raises(ValueError):
        oracle.labels_uf([-1], [0], 3)


def test_golden_fig1b():
    gold = json.load(open(os.path.join(GOLDEN, "fig1b_example.json")))
    lab = oracle.labels_uf(gold["edges_u"], gold["edges_v"], gold["n"])
    assert lab.tolist() == gold["expected_labels"]
    assert oracle.labels_bfs_brute(gold["edges_u"], gold["edges_v"], gold["n"]).tolist() == gold["expected_labels"]


# ------------------------------------------------- planted mistakes must fail
def _uf_variant(u, v, n, link_larger_root=False, no_final_find=False, skip_compress_check=False,
                drop_every_kth=0):
    p = list(range(n))

    def find(x):
        r = x
        while p[r] != r:
            r = p[r]
        while p[x] != r:
            p[x], x = r, p[x]
        return r

    for i, (a, b) in enumerate(zip(u, v)):
        if drop_every_kth and i % drop_every_kth == drop_every_kth - 1:
            continue
        ra, rb = find(a), find(b)
        if ra == rb:
            continue
        lo, hi = min(ra, rb), max(ra, rb)
        if link_larger_root:
            p[lo] = hi
        else:
            p[hi] = lo
    if no_final_find:
        return np.array(p, np.int32)
    return np.array([find(x) for x in range(n)], np.int32)


def _pins_pass(fn):
    """Run a candidate labelling function through a subset of the pins above."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = int(rng.integers(2, 10))
        m = int(rng.integers(0, 2 * n))
        u = rng.integers(0, n, m).tolist()
        v = rng.integers(0, n, m).tolist()
        if not np.array_equal(fn(u, v, n), oracle.labels_bfs_brute(u, v, n)):
            return False
    pi = gen.permutation(300, seed=1)
    if not np.all(fn(pi[:-1].tolist(), pi[1:].tolist(), 300) == 0):
        return False
    return True


def test_pins_accept_correct_variant():
    assert _pins_pass(lambda u, v, n: _uf_variant(u, v, n))


@pytest.mark.parametrize("kw", [dict(link_larger_root=True), dict(no_final_find=True),
                                dict(drop_every_kth=7)])
def test_pins_reject_planted_mistakes(kw):
    assert not _pins_pass(lambda u, v, n: _uf_variant(u, v, n, **kw))


# ------------------------------------------------------------ 64-bit ids
I64_MIN, I64_MAX = np.iinfo(np.int64).min, np.iinfo(np.int64).max


def _random_ids64(rng, k):
    """k distinct 64-bit ids spread over the whole range, extremes included."""
    pool = set([I64_MIN, I64_MAX, -1, 0, 1])
    while len(pool) < k + 5:
        pool.add(int(rng.integers(I64_MIN, I64_MAX, dtype=np.int64)))
    return np.asarray(rng.permutation(sorted(pool))[:k], dtype=np.int64)


def test_labels64_against_brute_force():
    rng = np.random.default_rng(64)
    for trial in range(200):
        k = int(rng.integers(1, 14))
        ids = _random_ids64(rng, k)
        m = int(rng.integers(0, 20))
        a = ids[rng.integers(0, k, m)]
        b = ids[rng.integers(0, k, m)]
        got = oracle.labels64(a, b)
        exp = oracle.labels64_brute(a, b)
        assert np.array_equal(got[0], exp[0]) and np.array_equal(got[1], exp[1]), trial


def test_labels64_reduces_to_dense_labels():
    """Ids 0 .. n-1 that all occur: the 64-bit labels are the dense ones."""
    g = gen.gnm(3000, 2500, seed=5)
    u = np.concatenate([g.u, np.arange(g.n, dtype=np.int32)])    # self-loops make every id occur
    v = np.concatenate([g.v, np.arange(g.n, dtype=np.int32)])
    ids, lab = oracle.labels64(u.astype(np.int64), v.astype(np.int64))
    assert np.array_equal(ids, np.arange(g.n))
    assert np.array_equal(lab, oracle.labels_uf(u, v, g.n).astype(np.int64))


def test_labels64_order_preserving_map_commutes():
    """An increasing map of the ids maps the labels the same way; a
    decreasing one turns each component's label into the image of its
    largest member."""
    g = gen.rmat(12, 4, seed=6)
    u, v = g.u.astype(np.int64), g.v.astype(np.int64)
    ids, lab = oracle.labels64(u, v)
    f = lambda x: x * 1_000_003 - (1 << 40)                      # increasing, no overflow here
    ids2, lab2 = oracle.labels64(f(u), f(v))
    assert np.array_equal(ids2, f(ids)) and np.array_equal(lab2, f(lab))
    ids3, lab3 = oracle.labels64(-u, -v)                         # decreasing
    big = {}
    for x, l in zip(ids.tolist(), lab.tolist()):
        big[l] = max(big.get(l, x), x)
    exp = {-x: -big[l] for x, l in zip(ids.tolist(), lab.tolist())}
    assert all(exp[x] == l for x, l in zip(ids3.tolist(), lab3.tolist()))


def test_labels64_planted_mistake_fails():
    """Numbering the ids in order of first appearance instead of sorted order
    (a relabel that does not keep the order) labels by the wrong member."""
    u = np.asarray([50, 7], dtype=np.int64)
    v = np.asarray([7, 50], dtype=np.int64)
    order = {50: 0, 7: 1}                                         # first appearance
    cu = np.asarray([order[x] for x in u.tolist()], np.int32)
    cv = np.asarray([order[x] for x in v.tolist()], np.int32)
    lab = oracle.labels_uf(cu, cv, 2)
    wrong = np.asarray([50, 7], np.int64)[lab]
    ids, exp = oracle.labels64_brute(u, v)
    assert not np.array_equal(np.sort(wrong), exp)
    assert np.array_equal(oracle.labels64(u, v)[1], exp)
