"""GPU parity of batched mode (one persistent launch for many graphs) against
the oracle run graph by graph, bit-exact."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")


def run_batch(b, **kw):
    say(f"[gpu] batched G={b.G} m={int(b.edge_off[-1])} n={int(b.vert_off[-1])} {kw}")
    return ccmi.label_batched(torch.from_numpy(np.ascontiguousarray(b.u)).cuda(),
                              torch.from_numpy(np.ascontiguousarray(b.v)).cuda(),
                              torch.from_numpy(b.edge_off).cuda(), torch.from_numpy(b.vert_off).cuda(), **kw)


def expected(b):
    parts = []
    for g in range(b.G):
        sub = b.graph(g)
        parts.append(oracle.labels_uf(sub.u, sub.v, sub.n))
    return np.concatenate(parts) if parts else np.zeros(0, np.int32)


def test_batch_small_families():
    b = gen.batch(64, 5_000_000, lg_hi=14.0)
    lab, st = run_batch(b, stats=True)
    say(f"   passes={st['passes']} blocks={st['blocks']} tile={st['tile_edges']} ms={st['ms_total']:.3f} "
        f"read={st['edges_read']} atomics={st['atomics']} chase={st['chase_reads']} kept={st['survivors_written']}")
    assert np.array_equal(lab.cpu().numpy(), expected(b))
    # the byte model's counts: the first pass reads every edge and later
    # passes read what earlier ones kept
    m = int(b.edge_off[-1])
    assert st["edges_read"] == m + st["survivors_written"]
    assert st["atomics"] > 0 and st["chase_reads"] >= 0


def test_batch_uneven_sizes():
    b = gen.batch(300, 7_000_000, lg_lo=4.0, lg_hi=17.0)
    lab = run_batch(b)
    assert np.array_equal(lab.cpu().numpy(), expected(b))


@pytest.mark.parametrize("tile", [1, 100, 4096, 1 << 20])
def test_explicit_tiles_agree(tile):
    b = gen.batch(40, 9_000_000, lg_hi=13.0)
    lab = run_batch(b, tile_edges=tile)
    assert np.array_equal(lab.cpu().numpy(), expected(b))


def _manual(graphs):
    us, vs, eo, vo = [], [], [0], [0]
    for u, v, n in graphs:
        us.append(np.asarray(u, np.int32))
        vs.append(np.asarray(v, np.int32))
        eo.append(eo[-1] + len(u))
        vo.append(vo[-1] + n)
    b = gen.Batch(np.concatenate(us) if us else np.zeros(0, np.int32),
                  np.concatenate(vs) if vs else np.zeros(0, np.int32),
                  np.array(eo, np.int64), np.array(vo, np.int64), np.zeros(len(graphs), np.int32))
    return b


def test_edge_cases():
    big = gen.rmat(16, 8, seed=3)
    graphs = [([], [], 0), ([], [], 1), ([0], [0], 1), ([], [], 5), ([1, 3], [2, 4], 5),
              (big.u, big.v, big.n), ([0, 1], [1, 0], 2), ([], [], 0)]
    b = _manual(graphs)
    assert np.array_equal(run_batch(b).cpu().numpy(), expected(b))
    # a single graph
    b1 = _manual([(big.u, big.v, big.n)])
    assert np.array_equal(run_batch(b1).cpu().numpy(), oracle.labels_uf(big.u, big.v, big.n))
    # only edgeless graphs
    b2 = _manual([([], [], 3), ([], [], 4)])
    assert np.array_equal(run_batch(b2).cpu().numpy(), np.array([0, 1, 2, 0, 1, 2, 3], np.int32))


def test_errors():
    b = _manual([([0, 1], [1, 2], 3), ([0], [3], 3)])      # local id 3 in a 3-vertex graph
    with pytest.raises(ccmi.CCError) as ei:
        run_batch(b)
    assert ei.value.code == ccmi.CC_ERANGE
    b = _manual([([0], [1], 2), ([0], [1], 2)])
    b.edge_off[:] = [0, 2, 1]                               # not non-decreasing... and edge_off[G] = 1
    with pytest.raises(ccmi.CCError) as ei:
        run_batch(b)
    assert ei.value.code == ccmi.CC_EINVAL
    b = _manual([([0], [1], 2)])
    b.vert_off[:] = [1, 3]
    with pytest.raises(ccmi.CCError) as ei:
        run_batch(b)
    assert ei.value.code == ccmi.CC_EINVAL


def test_repeatable_and_matches_single_calls():
    b = gen.batch(24, 11_000_000, lg_hi=15.0)
    first = run_batch(b)
    for _ in range(5):
        assert torch.equal(run_batch(b), first)
    # same labels as per-graph cc_label calls
    for g in range(b.G):
        sub = b.graph(g)
        if sub.n == 0:
            continue
        lab = ccmi.label(torch.from_numpy(np.ascontiguousarray(sub.u)).cuda(),
                         torch.from_numpy(np.ascontiguousarray(sub.v)).cuda(), sub.n, route="sv")
        a, c = int(b.vert_off[g]), int(b.vert_off[g + 1])
        assert torch.equal(lab, first[a:c])


def test_dense_and_deep_graphs():
    """Edge-heavy graphs (2m/n > 8, so the first pass runs in 8 pieces with a
    flatten after each) next to long permuted paths (deep trees)."""
    graphs = []
    for s in range(6):
        g = gen.rmat(13, 16, seed=40 + s)
        graphs.append((g.u, g.v, g.n))
        n = 20_000 + 997 * s
        pi = gen.permutation(n, seed=60 + s)
        graphs.append((pi[:-1], pi[1:], n))
    b = _manual(graphs)
    exp = expected(b)
    for kw in [{}, {"max_link": 1}, {"max_link": 4}, {"tile_edges": 1}]:
        assert np.array_equal(run_batch(b, **kw).cpu().numpy(), exp), kw


def test_large_mixed_batch():
    """A batch of 5.8 M edges: Kronecker graphs, G(n,m) graphs, ordered
    paths (ids and edge order follow the path: deep chains within the first
    pass) and permuted paths, every graph against the oracle, with the
    autotuned shape and with one hook attempt per pass; the byte model's
    read count covers every edge once plus the survivors."""
    graphs = []
    for s in range(3):
        g = gen.rmat(16, 16, seed=70 + s)
        graphs.append((g.u, g.v, g.n))
        g = gen.gnm(1 << 17, 3 << 17, seed=80 + s)
        graphs.append((g.u, g.v, g.n))
    for s in range(2):
        n = 400_000 + 1234 * s
        ids = np.arange(n, dtype=np.int32)
        graphs.append((ids[:-1], ids[1:], n))
        pi = gen.permutation(n, seed=90 + s)
        graphs.append((pi[:-1], pi[1:], n))
    b = _manual(graphs)
    m = int(b.edge_off[-1])
    assert m >= 1 << 22
    exp = expected(b)
    for kw in [{}, {"max_link": 1}]:
        lab, st = run_batch(b, stats=True, **kw)
        say(f"   passes={st['passes']} blocks={st['blocks']} chase={st['chase_reads']} ms={st['ms_total']:.3f}")
        assert st["blocks"] > 0
        assert np.array_equal(lab.cpu().numpy(), exp), kw
        assert st["edges_read"] == m + st["survivors_written"]


def test_barrier_timeout_falls_back_to_union(monkeypatch):
    """A grid barrier that waits past its spin limit (here forced from the
    host: a limit of one 100 MHz tick, so every early workgroup gives up and
    all exit) makes the call fall back to the disjoint-union SV loop: the
    labels are still exact and the stats report no persistent grid."""
    monkeypatch.setenv("CC_BATCH_BARRIER_TICKS", "1")
    b = gen.batch(40, 4_242_000, lg_hi=13.0)
    lab, st = run_batch(b, tile_edges=4096, max_link=1, stats=True)
    say(f"   passes={st['passes']} blocks={st['blocks']}")
    assert st["blocks"] == 0
    assert np.array_equal(lab.cpu().numpy(), expected(b))
    monkeypatch.delenv("CC_BATCH_BARRIER_TICKS")
    lab, st = run_batch(b, tile_edges=4096, max_link=1, stats=True)
    assert st["blocks"] > 0
    assert np.array_equal(lab.cpu().numpy(), expected(b))
