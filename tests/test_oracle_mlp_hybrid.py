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


# ------------------------------------------------------------ bfs_levels pins
# The level count of a BFS from s is the eccentricity of s within its
# component plus one (the last level finds nothing new).  Pinned against
# closed forms and a distance-by-distance brute force; an off-by-one variant
# must fail.

def _levels_brute(u, v, n, s):
    """Plain queue BFS with explicit distances: 1 + max distance from s."""
    from collections import deque
    if s < 0:
        return 0
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    dist = {s: 0}
    q = deque([s])
    while q:
        x = q.popleft()
        for y in adj[x]:
            if y not in dist:
                dist[y] = dist[x] + 1
                q.append(y)
    return 1 + max(dist.values())


def _grid_edges(L, perm):
    u, v = [], []
    for r in range(L):
        for c in range(L):
            x = r * L + c
            if c + 1 < L:
                u.append(perm[x]); v.append(perm[x + 1])
            if r + 1 < L:
                u.append(perm[x]); v.append(perm[x + L])
    return np.array(u), np.array(v)


def _levels_pins_pass(fn):
    n = 257
    pi = gen.permutation(n, seed=3)
    pu, pv = pi[:-1], pi[1:]                      # a path through every vertex
    if fn(pu, pv, n, int(pi[0])) != n:            # from one end: n levels
        return False
    if fn(pu, pv, n, int(pi[n // 2])) != n // 2 + 1:   # from the middle
        return False
    su = np.zeros(40, np.int64)
    sv = np.arange(1, 41)
    if fn(su, sv, 41, 0) != 2 or fn(su, sv, 41, 7) != 3:   # star: centre, leaf
        return False
    if fn(su, sv, 45, 43) != 1:                   # isolated seed
        return False
    L = 9
    perm = gen.permutation(L * L, seed=4)
    gu, gv = _grid_edges(L, perm)
    if fn(gu, gv, L * L, int(perm[0])) != 2 * L - 1:        # corner of a full grid
        return False
    if fn(gu, gv, L * L, int(perm[(L // 2) * L + L // 2])) != L:   # centre (L odd)
        return False
    rng = np.random.default_rng(9)
    for _ in range(40):
        nn = int(rng.integers(1, 40))
        mm = int(rng.integers(0, 2 * nn))
        u = rng.integers(0, nn, mm)
        v = rng.integers(0, nn, mm)
        s = int(rng.integers(0, nn))
        if fn(u, v, nn, s) != _levels_brute(u, v, nn, s):
            return False
    return True


def test_bfs_levels_pins():
    assert hybrid.bfs_levels(np.zeros(0, np.int64), np.zeros(0, np.int64), 5, -1) == 0
    assert _levels_pins_pass(hybrid.bfs_levels)


def test_bfs_levels_pins_reject_off_by_one():
    # counting only the levels that discover a vertex (the eccentricity) must fail
    assert not _levels_pins_pass(lambda u, v, n, s: hybrid.bfs_levels(u, v, n, s) - 1)
    assert not _levels_pins_pass(lambda u, v, n, s: hybrid.bfs_levels(u, v, n, s) + 1)


# ------------------------------------------------------- router_features pins
# Hand-computed feature vector: n = 1024 vertices, m = 4096 edges, with 24
# isolated vertices (bin 0), 500 of degree 2 (bin 3), 400 of degree 4 or 5
# (bin 5) and 100 of degree 8..11 (bin 7).  Every fraction is exact in binary.
_HAND_LOG64 = {0: 24, 3: 500, 5: 400, 7: 100}
_HAND_FEATURES = [0.0] * 66
_HAND_FEATURES[0] = 0.0234375      # 24 / 1024
_HAND_FEATURES[3] = 0.48828125     # 500 / 1024
_HAND_FEATURES[5] = 0.390625       # 400 / 1024
_HAND_FEATURES[7] = 0.09765625     # 100 / 1024
_HAND_FEATURES[64] = 10.0          # log2 1024
_HAND_FEATURES[65] = 12.0          # log2 4096


def _hand_log64():
    h = np.zeros(64, np.int64)
    for k, c in _HAND_LOG64.items():
        h[k] = c
    return h


def test_router_features_hand_computed():
    f = odeg.router_features(_hand_log64(), 1024, 4096)
    assert f.shape == (66,)
    assert f.tolist() == _HAND_FEATURES


def test_router_features_from_degree_sequence():
    # the same histogram reached from a concrete degree sequence through log_bins
    deg = np.concatenate([np.zeros(24), np.full(500, 2), np.full(200, 4), np.full(200, 5),
                          np.full(50, 8), np.full(50, 11)]).astype(np.int64)
    log64, _, _ = odeg.histograms(deg)
    assert odeg.router_features(log64, 1024, 4096).tolist() == _HAND_FEATURES
    # degenerate sizes: log2 of max(., 1)
    f0 = odeg.router_features(np.zeros(64, np.int64), 0, 0)
    assert f0[64] == 0.0 and f0[65] == 0.0 and not f0[:64].any()


def test_router_features_pin_rejects_natural_log():
    def ln_variant(log64, n, m):
        f = odeg.router_features(log64, n, m)
        f[64], f[65] = np.log(max(n, 1)), np.log(max(m, 1))
        return f

    def unnormalised_variant(log64, n, m):
        f = odeg.router_features(log64, n, m)
        f[:64] = np.asarray(log64, np.float64)
        return f

    for bad in (ln_variant, unnormalised_variant):
        assert bad(_hand_log64(), 1024, 4096).tolist() != _HAND_FEATURES
