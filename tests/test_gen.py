"""The seeded generators: determinism, exact sizes, bijective permutations."""
import numpy as np

import gen


def test_deterministic():
    a = gen.rmat(12, 8, seed=5)
    b = gen.rmat(12, 8, seed=5)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v)
    c = gen.rmat(12, 8, seed=6)
    assert not np.array_equal(a.u, c.u)


def test_gnm_simple_graph():
    g = gen.gnm(1000, 3000, seed=1)
    assert g.m == 3000 and np.all(g.u != g.v)
    key = np.minimum(g.u, g.v).astype(np.int64) * 1000 + np.maximum(g.u, g.v)
    assert np.unique(key).shape[0] == 3000


def test_grid_sizes_and_permutation():
    g = gen.grid(64, 1.0, seed=1)
    assert g.m == 2 * 64 * 63 and g.u.max() < 64 * 64
    p = gen.permutation(100_000, seed=3)
    assert np.array_equal(np.sort(p), np.arange(100_000))


def test_plcomp_degree_cap_and_size():
    g = gen.plcomp(200_000, seed=2)
    deg = np.bincount(np.concatenate([g.u, g.v]), minlength=g.n)
    assert deg.max() <= 8
    assert 1.1 < g.m / g.n < 1.4
    s = gen.plcomp_sizes(200_000, seed=2)
    assert s.sum() == 200_000 and s.max() <= 100_000


def test_batch_layout():
    b = gen.batch(16, 5_000_000, lg_hi=12.0)
    assert b.G == 16 and b.edge_off[-1] == b.u.shape[0]
    for g in range(b.G):
        sub = b.graph(g)
        if sub.m:
            assert sub.u.max() < sub.n and sub.v.max() < sub.n and min(sub.u.min(), sub.v.min()) >= 0
