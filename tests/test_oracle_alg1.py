"""Pins for the Algorithm 1 transcription: the worked example's notation values,
agreement with brute force / union-find, and the logarithmic iteration count."""
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import alg1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_notation():
    gold = json.load(open(os.path.join(GOLDEN, "fig1b_example.json")))
    a = gold["assignment"]
    p, q, r = alg1.initial_tuples(gold["edges_u"], gold["edges_v"], gold["n"])
    assert sorted(alg1.partitions(p)) == gold["P0"]
    assert sorted(t[0] for t in alg1.vertex_bucket(p, q, r, a["u"])) == gold["VB0_u_partitions"]
    assert all(t[2] == a["u"] for t in alg1.vertex_bucket(p, q, r, a["u"]))
    pb = alg1.partition_bucket(p, q, r, a["u"])
    assert all(t[0] == a["u"] for t in pb)
    assert sorted(t[2] for t in pb) == gold["PB0_u_vertices"]
    assert sorted(alg1.neighborhood(p, r, a["v1"])) == gold["N0_v1"]
    lab, _ = alg1.run(gold["edges_u"], gold["edges_v"], gold["n"])
    assert lab.tolist() == gold["expected_labels"]


@pytest.mark.parametrize("exclude", [False, True])
def test_alg1_matches_brute_force_small(exclude):
    rng = np.random.default_rng(3)
    for _ in range(300):
        n = int(rng.integers(1, 14))
        m = int(rng.integers(0, 3 * n))
        u = rng.integers(0, n, m)
        v = rng.integers(0, n, m)
        lab, _ = alg1.run(u, v, n, exclude_completed=exclude)
        assert np.array_equal(lab, oracle.labels_bfs_brute(u, v, n))


@pytest.mark.parametrize("exclude", [False, True])
def test_alg1_matches_uf_medium(exclude):
    for seed, g in enumerate([gen.gnm(1000, 900, seed=1), gen.rmat(10, 4, seed=2),
                              gen.grid(30, 0.6, seed=3), gen.plcomp(1000, seed=4)]):
        lab, _ = alg1.run(g.u, g.v, g.n, exclude_completed=exclude)
        assert np.array_equal(lab, oracle.labels_uf(g.u, g.v, g.n)), g.name


def test_alg1_logarithmic_iterations_on_paths():
    """Section III-A.2: pointer doubling gives O(log n) iterations where plain
    min-propagation would need O(n) on a path."""
    for n in [64, 256, 1024, 4096]:
        pi = gen.permutation(n, seed=n)
        lab, it = alg1.run(pi[:-1], pi[1:], n)
        assert np.all(lab == 0)
        assert it <= 3 * math.ceil(math.log2(n)) + 2, (n, it)


def test_alg1_excluding_completed_shrinks_work():
    """Section III-A.4: completed partitions leave the working set; labels unchanged."""
    g = gen.plcomp(5000, seed=9)
    a, _ = alg1.run(g.u, g.v, g.n, exclude_completed=False)
    b, _ = alg1.run(g.u, g.v, g.n, exclude_completed=True)
    assert np.array_equal(a, b)
