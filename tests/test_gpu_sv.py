"""GPU parity of the SV routes (R1 plain SV, R2 SV-theta, and R1 chosen after
the degree pass) against the oracle, bit-exact."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev

pytestmark = pytest.mark.gpu

ccmi = pytest.importorskip("paper_1607_06156_amd")
ROUTES = ["sv", "sv-theta", "predicted-sv"]


def run(g, route, **kw):
    say(f"[gpu] {g.name} m={g.m} n={g.n} route={route}")
    if route == "predicted-sv":
        # degree pass and power-law fit first, then SV (tau below any K-S value)
        route, kw = "heuristic", dict(kw, tau=1e-300)
    return ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route=route, **kw)


def test_predicted_sv_route_taken():
    g = gen.workload("rmat16")
    lab, st = run(g, "predicted-sv", stats=True)
    assert st["route"] == 1 and st["max_degree"] > 0   # R1 after the degree pass
    assert_labels_equal(lab, oracle_labels(g), "rmat16/predicted-sv")


@pytest.mark.parametrize("route", ROUTES)
def test_sparse_buckets_and_hubs(route):
    """Ids spread over many 2^15-vertex buckets, most of them empty; a hub
    with most edges; loops and duplicates only in the last bucket."""
    rng = np.random.default_rng(11)
    n = 3_000_017
    u = rng.integers(0, n, 5000).astype(np.int32)
    v = rng.integers(0, n, 5000).astype(np.int32)
    g = gen.Graph(u, v, n, "sparse-buckets")
    assert_labels_equal(run(g, route), oracle_labels(g), g.name)
    leaves = rng.integers(0, n, 200_000).astype(np.int32)
    hub = np.full(leaves.size, 2_999_999, np.int32)
    g = gen.Graph(np.concatenate([hub, leaves[:100]]), np.concatenate([leaves, leaves[:100]]), n, "hub")
    assert_labels_equal(run(g, route), oracle_labels(g), g.name)
    tail = np.arange(n - 40, n, dtype=np.int32)
    g = gen.Graph(np.concatenate([tail, tail[:-1]]), np.concatenate([tail, tail[1:]]), n, "last-bucket")
    assert_labels_equal(run(g, route), oracle_labels(g), g.name)


@pytest.mark.parametrize("route", ROUTES)
def test_closed_forms(route):
    n = 40_000
    pi = gen.permutation(n, seed=1)
    # Hamiltonian path, ids permuted -> one component
    lab = run(gen.Graph(pi[:-1], pi[1:], n, "path"), route)
    assert torch.all(lab == 0)
    # complete grid -> one component
    lab = run(gen.grid(150, 1.0, seed=2), route)
    assert torch.all(lab == 0)
    # no edges -> identity
    e = np.zeros(0, np.int32)
    lab = run(gen.Graph(e, e, 1000, "empty"), route)
    assert torch.equal(lab.cpu(), torch.arange(1000, dtype=torch.int32))
    # perfect matching
    a = np.arange(0, n, 2, dtype=np.int32)
    lab = run(gen.Graph(a + 1, a, n, "matching"), route)
    assert torch.equal(lab.cpu(), torch.from_numpy(2 * (np.arange(n, dtype=np.int32) // 2)))
    # self-loops only
    x = np.arange(777, dtype=np.int32)
    lab = run(gen.Graph(x, x, 777, "loops"), route)
    assert torch.equal(lab.cpu(), torch.from_numpy(x))
    # star
    leaves = np.array([y for y in range(5000) if y != 1234], np.int32)
    lab = run(gen.Graph(np.full(4999, 1234, np.int32), leaves, 5000, "star"), route)
    assert torch.all(lab == 0)


@pytest.mark.parametrize("route", ROUTES)
def test_random_small_multigraphs(route):
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 3 * n))
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        if m and trial % 3 == 0:
            v[: m // 4] = u[: m // 4]
        g = gen.Graph(u, v, n, f"rand{trial}")
        assert_labels_equal(run(g, route), oracle_labels(g), g.name)


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("name", ["gnm64k", "rmat16", "grid512", "plcomp1m", "rmat18noisy"])
def test_workloads_small(route, name):
    g = gen.workload(name)
    lab, st = run(g, route, stats=True)
    assert_labels_equal(lab, oracle_labels(g), f"{name}/{route}")
    say(f"   passes={st['sv_passes']} active={st['active_edges'][:8]} ms={st['ms_total']:.3f}")
    # the active set never grows and the loop ends with no active edge
    act = st["active_edges"]
    assert all(b <= a for a, b in zip(act, act[1:]))


@pytest.mark.parametrize("route", ROUTES)
def test_ragged_sizes(route):
    """m not a multiple of the tile, a few edges per block, one block."""
    for m in [1, 3, 5, 1023, 1025, 4097, 70001]:
        g = gen.gnm(max(8, m), m, seed=m)
        assert_labels_equal(run(g, route), oracle_labels(g), f"gnm m={m}")


def test_edge_order_and_orientation_invariance():
    g = gen.rmat(15, 8, seed=3)
    rng = np.random.default_rng(0)
    order = rng.permutation(g.m)
    swap = rng.random(g.m) < 0.5
    g2 = gen.Graph(np.where(swap, g.v, g.u)[order], np.where(swap, g.u, g.v)[order], g.n, "shuffled")
    a = run(g, "sv")
    b = run(g2, "sv")
    assert torch.equal(a, b)


def test_repeatable():
    g = gen.workload("rmat16")
    first = run(g, "sv")
    for _ in range(10):
        assert torch.equal(run(g, "sv"), first)


def test_errors():
    u = to_dev(np.array([0, 5], np.int32))
    v = to_dev(np.array([1, 2], np.int32))
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(u, v, 5, route="sv")
    assert ei.value.code == ccmi.CC_ERANGE
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(u, v, -1, route="sv", out=torch.empty(1, dtype=torch.int32, device="cuda"))
    assert ei.value.code == ccmi.CC_EINVAL
    neg = to_dev(np.array([-3], np.int32))
    with pytest.raises(ccmi.CCError):
        ccmi.label(neg, neg, 4, route="sv")
    # m = 0 -> identity, n = 0 -> nothing to do
    e = to_dev(np.zeros(0, np.int32))
    assert torch.equal(ccmi.label(e, e, 9, route="sv").cpu(), torch.arange(9, dtype=torch.int32))
    assert ccmi.label(e, e, 0, route="sv").numel() == 0


def test_pass_cap_reports_internal_error():
    n = 100_000
    pi = gen.permutation(n, seed=5)
    u, v = to_dev(pi[:-1]), to_dev(pi[1:])
    with pytest.raises(ccmi.CCError) as ei:
        ccmi.label(u, v, n, route="sv", max_passes=1)
    assert ei.value.code == ccmi.CC_EINTERNAL
    assert torch.all(ccmi.label(u, v, n, route="sv") == 0)


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("name,drops", [("rmat18", True), ("rmat18noisy", True), ("grid2048", None),
                                        ("plcomp4m", False)])
def test_largest_tree_bitmap(route, name, drops):
    """Lists long enough for a chunked first pass (m >= 2^22): after each
    flatten the largest tree's bitmap lets the next chunk drop the edges
    inside it.  R-MAT graphs drop most of their later chunks that way; a
    forest of small components has no tree holding 1/16 of the vertices and
    drops nothing.  Labels are exact either way, and the byte counters add
    up (every atomic issued is a hook, a failed hook or a retry).  With the
    degrees known (predicted-sv), the R-MAT hubs' probes come from the LDS
    table; the other routes list no hubs, nor does the lattice (no degree
    reaches the hub minimum)."""
    if name == "grid2048":
        g = gen.grid(2048, 0.7, seed=5)
    elif name == "plcomp4m":
        g = gen.plcomp(4_000_000, seed=6)
    else:
        g = gen.workload(name)
    lab, st = run(g, route, stats=True)
    assert_labels_equal(lab, oracle_labels(g), f"{name}/{route}")
    say(f"   dropped={st['giant_dropped']} of m={g.m} atomics={st['sv_atomics']} hooks={st['hooks_total']} "
        f"chase={st['sv_chase_reads']} ms={st['ms_total']:.3f}")
    if drops is True:
        assert st["giant_dropped"] > g.m // 2
    elif drops is False:
        assert st["giant_dropped"] == 0
    assert st["sv_atomics"] >= st["hooks_total"]
    if route == "predicted-sv" and drops is True:
        assert 0 < st["sv_hubs"] <= 2048
    elif route != "predicted-sv" or name == "grid2048":
        assert st["sv_hubs"] == 0



def test_hub_table_full_bucket():
    """R-MAT scale 18 with its twelve highest-degree vertices renamed to ids
    that share one bucket of the LDS hub table (a bucket holds four ids): the
    hubs left out of the table are probed in the largest tree's bitmap
    instead.  The list (2^22 edges) gets a chunked first pass, and the
    largest tree drops most later edges, so the table is in use.  Labels
    exact against the oracle."""
    g0 = gen.workload("rmat18")
    n = g0.n
    xs = np.arange(n, dtype=np.uint64)
    bucket = ((xs * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)) >> np.uint64(22)
    same = np.flatnonzero(bucket == 0)[:12]
    deg = np.bincount(g0.u, minlength=n) + np.bincount(g0.v, minlength=n)
    top = np.argsort(-deg, kind="stable")[:12]
    f = np.arange(n, dtype=np.int64)   # a permutation of the ids: swap each top vertex with a shared-bucket id
    for a, b in zip(top, same):
        ia, ib = np.flatnonzero(f == a)[0], np.flatnonzero(f == b)[0]
        f[ia], f[ib] = b, a
    new_top = f[top]
    assert int(np.sum(bucket[new_top] == 0)) >= 8
    g = gen.Graph(f[g0.u].astype(np.int32), f[g0.v].astype(np.int32), n, "rmat18, top hubs in one bucket")
    lab, st = run(g, "predicted-sv", stats=True)
    assert st["route"] == ccmi.R1_SV and 12 <= st["sv_hubs"] <= 2048
    assert st["giant_dropped"] > g.m // 2
    assert_labels_equal(lab, oracle_labels(g), g.name)


@pytest.mark.parametrize("name,tau,taken", [("rmat18", 1e-300, 1), ("rmat18", 1.0, 0), ("grid2048", 1e-300, 1)])
def test_first_launch_ahead_of_the_decision(name, tau, taken):
    """On lists cut into several first-pass chunks (m >= 2^22) the SV
    route's first launch is enqueued behind the degree pass, before the host
    has fitted the degree distribution (the fit runs on a second stream
    beside it).  Taking R1 goes on from that launch (not repeating it);
    taking R0 resets the forest and runs the BFS route.  Labels are exact
    either way, on a dense list (first launch 1/64 of the edges) and a
    sparse one (the whole first chunk).  The lattice's degrees leave the
    power-law fit no candidate cutoff, so no tau sends it to R0."""
    g = gen.workload(name) if name != "grid2048" else gen.grid(2048, 0.7, seed=5)
    assert g.m >= 1 << 22
    say(f"[gpu] {g.name} m={g.m} tau={tau}")
    for scratch in ("cached", "pool"):
        lab, st = ccmi.label(to_dev(g.u), to_dev(g.v), g.n, route="heuristic", tau=tau, stats=True, profile=True,
                             scratch=scratch)
        assert st["route"] == taken
        assert_labels_equal(lab, oracle_labels(g), f"{g.name}/tau={tau}/{scratch}")
        assert st["ms_predict"] > 0 and st["ms_sv"] > 0
        if taken == 1:
            # R1's passes each take at least one launch, the first pass several
            k = ccmi.KERNEL_CLASSES.index("sv_pass")
            assert st["kernel_launches"][k] >= st["sv_passes"] + 1
