"""Full-size workloads on the GPU, checked against the oracle: the near-critical
G(n,m), R-MAT scale 24 (plain, and with per-level noise: the heuristic takes
the BFS route), the 8192^2 thinned lattice and the 200M-vertex component
forest (also through the BFS route, whose remaining list is long, and through
the learned router) label for label; the 4096-graph batch graph by graph,
every graph against the oracle."""
import os
from concurrent.futures import ThreadPoolExecutor

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
    ("grid8192", ["sv", "sv-theta", "heuristic"]),
    ("plcomp200m", ["sv", "heuristic", "bfs+sv", "router"]),
])
def test_full_workload(name, routes):
    g, expect = workload(name)
    u, v = to_dev(g.u), to_dev(g.v)
    for r in routes:
        if r == "router":
            ccmi.router_load(os.path.join(os.path.dirname(ccmi.__file__), "router_weights.txt"))
        try:
            lab, st = ccmi.label(u, v, g.n, route=r, stats=True)
        finally:
            if r == "router":
                ccmi.router_set(None)
        say(f"   {name}/{r}: took {st['route_name']} passes={st['sv_passes']} ks={st['ks_statistic']:.4g} "
            f"ms={st['ms_total']:.2f}")
        assert_labels_equal(lab, expect, f"{name}/{r}")
        del lab
    del u, v
    torch.cuda.empty_cache()


def oracle_batch(b, workers=None):
    """Oracle labels of every graph of a batch, concatenated; the graphs run
    on a thread pool (the oracle's C union-find releases the GIL)."""
    workers = workers or min(16, os.cpu_count() or 1)
    out = np.empty(int(b.vert_off[-1]), dtype=np.int32)

    def one(g):
        sub = b.graph(g)
        a = int(b.vert_off[g])
        out[a:a + sub.n] = oracle.labels_uf(sub.u, sub.v, sub.n)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, range(b.G)))
    return out


def test_full_batch_every_graph():
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
    del lab, u, v, eo, vo
    torch.cuda.empty_cache()
    say(f"[gpu] oracle over all {b.G} graphs")
    expect = oracle_batch(b)
    if not np.array_equal(lab_h, expect):
        bad = np.flatnonzero(lab_h != expect)
        graphs = np.unique(np.searchsorted(b.vert_off, bad, side="right") - 1)
        raise AssertionError(f"{bad.size} labels differ, in graphs {graphs[:10].tolist()}")
