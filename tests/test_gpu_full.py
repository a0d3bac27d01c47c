"""Full-size workloads on the GPU, checked against the oracle: the near-critical
G(n,m), R-MAT scale 24 (plain, and with per-level noise: the heuristic takes
the BFS route), the 8192^2 thinned lattice and the 200M-vertex component
forest (also through the BFS route, whose remaining list is long) label for
label; the 4096-graph batch on sampled graphs plus invariants over every
graph."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_labels_equal, say, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
ccmi = pytest.importorskip("paper_1607_06156_amd")

_cache = {}


def workload(name):
    if name not in _cache:
        _cache.clear()
        say(f"[gpu] generating {name}")
        g = gen.workload(name)
        say(f"[gpu] oracle {name} m={g.m} n={g.n}")
        _cache[name] = (g, oracle.labels_uf(g.u, g.v, g.n))
    return _cache[name]


@pytest.mark.parametrize("name,routes", [
    ("gnm64k", ["sv", "sv-theta", "bfs+sv", "heuristic"]),
    ("rmat24", ["heuristic", "sv", "bfs+sv", "sv-theta"]),
    ("rmat24noisy", ["heuristic", "sv"]),
    ("grid8192", ["sv", "sv-theta"]),
    ("plcomp200m", ["sv", "heuristic", "bfs+sv"]),
])
def test_full_workload(name, routes):
    g, expect = workload(name)
    u, v = to_dev(g.u), to_dev(g.v)
    for r in routes:
        lab, st = ccmi.label(u, v, g.n, route=r, stats=True)
        say(f"   {name}/{r}: took {st['route_name']} passes={st['sv_passes']} ks={st['ks_statistic']:.4g} "
            f"ms={st['ms_total']:.2f}")
        assert_labels_equal(lab, expect, f"{name}/{r}")
        del lab
    del u, v
    torch.cuda.empty_cache()


def test_full_batch_sampled():
    say("[gpu] generating batch4096")
    b = gen.workload("batch4096")
    u = torch.from_numpy(b.u).cuda()
    v = torch.from_numpy(b.v).cuda()
    eo = torch.from_numpy(b.edge_off).cuda()
    vo = torch.from_numpy(b.vert_off).cuda()
    lab, st = ccmi.label_batched(u, v, eo, vo, stats=True)
    say(f"   batch4096: m={st['total_edges']} n={st['total_vertices']} passes={st['passes']} "
        f"blocks={st['blocks']} ms={st['ms_total']:.2f}")
    lab_h = lab.cpu().numpy()
    # oracle on a sample of graphs: every 64th, plus the largest
    gs = list(range(0, b.G, 64)) + [int(np.argmax(np.diff(b.edge_off)))]
    for g in gs:
        sub = b.graph(g)
        a, c = int(b.vert_off[g]), int(b.vert_off[g + 1])
        assert np.array_equal(lab_h[a:c], oracle.labels_uf(sub.u, sub.v, sub.n)), f"graph {g}"
    # invariants over every graph, on the device: endpoints share a label,
    # label <= local id, labels are fixed points
    gid_e = torch.repeat_interleave(torch.arange(b.G, device="cuda"), torch.diff(eo))
    base_e = vo[gid_e]
    lu = lab[(u.long() + base_e)]
    lv = lab[(v.long() + base_e)]
    assert torch.equal(lu, lv)
    gid_v = torch.repeat_interleave(torch.arange(b.G, device="cuda"), torch.diff(vo))
    local = torch.arange(lab.numel(), device="cuda") - vo[gid_v]
    assert bool(torch.all(lab.long() <= local))
    assert torch.equal(lab[(lab.long() + vo[gid_v])], lab)
