"""GPU parity on graphs whose first pass links long chains: paths and lattices
whose ids and edge order both follow the graph, so that a pass hooks every
vertex onto its predecessor at once.  Every walk up the parent forest stops
after 64 links (an edge whose find stopped there is kept as the pair of
ancestors reached), and flatten rounds finish the chains; without the bound
the finds and the final labelling of a chain of length L would cost O(L^2)
dependent loads.  Labels are exact; closed forms where the graph has one,
else the oracle."""
import numpy as np
import pytest
import torch

import gen
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")

ROUTES = ["sv", "sv-theta", "heuristic"]   # the forced BFS route on a long path: test_forced_bfs_on_a_long_path
CAP = 200                                  # SV passes: a runaway loop fails fast instead of spinning


def _label(u, v, n, route):
    return ccmi.label(to_dev(u), to_dev(v), n, route=route, stats=True, max_passes=CAP)


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("n", [100_000, 3_000_000])
def test_ordered_path(n, route):
    """Edge i joins i and i + 1, in that order: one component, label 0."""
    u = np.arange(n - 1, dtype=np.int32)
    say(f"[gpu] ordered path n={n} {route}")
    lab, st = _label(u, u + 1, n, route)
    assert torch.all(lab == 0), f"{int((lab != 0).sum())} labels differ from 0"
    say(f"   passes={st['sv_passes']} deep_rounds={st['sv_deep_rounds']} ms={st['ms_total']:.2f}")
    if n >= 1_000_000:
        assert st["sv_deep_rounds"] > 0      # the chain outgrew one walk


@pytest.mark.parametrize("route", ROUTES)
def test_ordered_paths_reversed_and_split(route):
    """Descending edge order, and 8 ordered paths side by side: label = the
    first vertex of each path."""
    n = 2_000_000
    x = np.arange(n - 1, 0, -1, dtype=np.int32)
    say(f"[gpu] reversed path {route}")
    lab, _ = _label(x, x - 1, n, route)
    assert torch.all(lab == 0)
    k = n // 8
    u = np.arange(n - 1, dtype=np.int32)
    keep = (u + 1) % k != 0                   # cut after every k-th vertex
    say(f"[gpu] split paths {route}")
    lab, _ = _label(u[keep], u[keep] + 1, n, route)
    assert torch.equal(lab.cpu(), torch.from_numpy((np.arange(n, dtype=np.int32) // k) * k))


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("p", [1.0, 0.7])
def test_ordered_lattice(route, p):
    """Row-major ids, edges in generation order."""
    g = gen.grid(1500, p, seed=9, permute=False, shuffle=False)
    say(f"[gpu] ordered lattice p={p} n={g.n} m={g.m} {route}")
    lab, st = _label(g.u, g.v, g.n, route)
    if p == 1.0:
        assert torch.all(lab == 0)
    else:
        assert_labels_equal(lab, oracle_labels(g), f"ordered lattice/{route}")
    say(f"   passes={st['sv_passes']} deep_rounds={st['sv_deep_rounds']}")


def test_ordered_paths_batched():
    """A batch of ordered paths (2^8 .. 2^18 vertices, graph-local ids) and
    ordered lattices: every path is one component (local label 0)."""
    rng = np.random.default_rng(10)
    us, vs, eo, vo, exp = [], [], [0], [0], []
    for k in range(48):
        if k % 6 == 5:
            g = gen.grid(int(rng.integers(40, 300)), 0.8, seed=k, permute=False, shuffle=False)
            u, v, n = g.u, g.v, g.n
            exp.append(oracle_labels(g))
        else:
            n = int(2 ** rng.uniform(8, 18))
            u = np.arange(n - 1, dtype=np.int32)
            v = u + 1
            if k % 2:
                u, v = v[::-1].copy(), u[::-1].copy()
            exp.append(np.zeros(n, np.int32))
        us.append(u)
        vs.append(v)
        eo.append(eo[-1] + u.size)
        vo.append(vo[-1] + n)
    args = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
            for a in (np.concatenate(us), np.concatenate(vs), np.array(eo, np.int64), np.array(vo, np.int64))]
    say(f"[gpu] batched ordered paths: {len(exp)} graphs, {vo[-1]} vertices")
    lab, st = ccmi.label_batched(*args, stats=True)
    assert np.array_equal(lab.cpu().numpy(), np.concatenate(exp))
    say(f"   passes={st['passes']} blocks={st['blocks']}")


@pytest.mark.parametrize("permute", [False, True])
def test_forced_bfs_on_a_long_path(permute):
    """The BFS step is for short-diameter components: on a 3M-vertex path it
    stops after 256 levels, before writing any label, and SV labels the
    whole graph (route reported R1)."""
    n = 3_000_000
    order = gen.permutation(n, seed=12) if permute else np.arange(n, dtype=np.int32)
    u, v = order[:-1].astype(np.int32), order[1:].astype(np.int32)
    say(f"[gpu] forced bfs+sv on a {'permuted' if permute else 'ordered'} path n={n}")
    lab, st = _label(u, v, n, "bfs+sv")
    assert torch.all(lab == 0)
    assert st["route"] == ccmi.R1_SV and st["bfs_levels"] == 256
    say(f"   bfs_visited={st['bfs_visited']} ms={st['ms_total']:.1f}")


def test_router_on_an_ordered_path():
    """With the shipped router weights, route "router" on a 3M-vertex ordered
    path: whichever route the MLP picks (a BFS is abandoned after 256 levels),
    the labels are exact."""
    import os
    weights = os.path.join(os.path.dirname(ccmi.__file__), "router_weights.txt")
    n = 3_000_000
    u = np.arange(n - 1, dtype=np.int32)
    ccmi.router_load(weights)
    try:
        say("[gpu] router on an ordered path")
        lab, st = _label(u, u + 1, n, "router")
    finally:
        ccmi.router_set(None)
    assert torch.all(lab == 0)
    say(f"   route={st['route_name']} bfs_levels={st['bfs_levels']} deep_rounds={st['sv_deep_rounds']}")
