"""Pins for the MLP reference (finite differences, closed form, descent) and for
the BFS-route reference of Algorithm 2 (visited set = component of the seed;
BFS step + SV on the rest reproduces the full labelling)."""
import numpy as np

import gen
import oracle
from oracle import degree as odeg
from oracle import hybrid, mlp


def test_mlp_zero_weights_closed_form():
    params = [np.zeros_like(p) for p in mlp.init_params(0)]
    params[5] = np.array([0.5, -1.0, 2.0])
    x = np.random.default_rng(0).random((4, 66))
    z, _ = mlp.forward(params, x)
    assert np.allclose(z, params[5])
    loss, _ = mlp.loss_and_grads([np.zeros_like(p) for p in params], x, np.array([0, 1, 2, 0]))
    assert abs(loss - np.log(3.0)) < 1e-15


def test_mlp_gradients_vs_finite_differences():
    rng = np.random.default_rng(1)
    params = mlp.init_params(3)
    x = rng.random((8, 66))
    y = rng.integers(0, 3, 8)
    _, grads = mlp.loss_and_grads(params, x, y)
    for pi, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.shape[0], size=min(12, flat.shape[0]), replace=False):
            h = 1e-6
            pp = [q.copy() for q in params]
            pp[pi].reshape(-1)[idx] += h
            lp, _ = mlp.loss_and_grads(pp, x, y)
            pp[pi].reshape(-1)[idx] -= 2 * h
            lm, _ = mlp.loss_and_grads(pp, x, y)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[pi].reshape(-1)[idx]) < 1e-6, (pi, idx)


def test_mlp_sgd_descends():
    rng = np.random.default_rng(2)
    x = rng.random((256, 66))
    y = (x[:, 0] > 0.5).astype(np.int64) + (x[:, 1] > 0.7)
    params = mlp.init_params(4)
    l0, _ = mlp.loss_and_grads(params, x, y)
    for _ in range(300):
        _, g = mlp.loss_and_grads(params, x, y)
        params = mlp.sgd_step(params, g, 0.1)
    l1, _ = mlp.loss_and_grads(params, x, y)
    assert l1 < 0.6 * l0


def test_seed_choice_ties_smallest_id():
    deg = np.array([3, 7, 2, 7, 7])
    assert hybrid.choose_seed(deg) == 1
    assert hybrid.choose_seed(np.zeros(4)) == -1


def test_bfs_visited_is_component_of_seed():
    for g in [gen.rmat(14, 8, seed=5), gen.gnm(30_000, 20_000, seed=6), gen.grid(150, 0.6, seed=7),
              gen.plcomp(40_000, seed=8)]:
        lab = oracle.labels_uf(g.u, g.v, g.n)
        deg = odeg.degree(g.u, g.v, g.n)
        s = hybrid.choose_seed(deg)
        vis = hybrid.bfs_visited(g.u, g.v, g.n, s)
        assert np.array_equal(vis, lab == lab[s]), g.name


def test_bfs_step_then_sv_reproduces_labels():
    """Algorithm 2 end to end: BFS component gets its minimum id, the filtered
    remainder is labelled separately, and together they equal the full labels."""
    for g in [gen.rmat(13, 16, seed=1), gen.gnm(5000, 6000, seed=2)]:
        r = hybrid.bfs_route(g.u, g.v, g.n)
        rest = oracle.labels_uf(r["u"], r["v"], g.n)
        combined = np.where(r["visited"], r["label"], rest)
        assert np.array_equal(combined, oracle.labels_uf(g.u, g.v, g.n))
        # filtered edges touch no visited vertex at either end
        assert not r["visited"][r["u"]].any() and not r["visited"][r["v"]].any()
