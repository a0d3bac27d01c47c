"""GPU parity of cc_label64 (arbitrary 64-bit vertex ids, relabelled on the
device) against the oracle's sorted relabel + union-find, bit-exact."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")

I64_MIN, I64_MAX = np.iinfo(np.int64).min, np.iinfo(np.int64).max


def mix_ids(x, salt):
    """A bijective 64-bit mix of the ids (odd multiply, xor-shifts), the kind
    of hash the paper applies to permute its 64-bit ids."""
    z = np.asarray(x, dtype=np.uint64) + np.uint64(salt)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(31))) * np.uint64(0x7FB5D329728EA185)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x81DADEF4BC2DD44D)
        z = z ^ (z >> np.uint64(33))
    return z.view(np.int64)


def check(u64, v64, route=None, n_max=0):
    u = torch.from_numpy(np.ascontiguousarray(u64)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(v64)).cuda()
    ids, lab, st = ccmi.label64(u, v, n_max=n_max, route=route, stats=True)
    ids = ids.cpu().numpy()
    lab = lab.cpu().numpy()
    order = np.argsort(ids, kind="stable")
    exp_ids, exp_lab = oracle.labels64(u64, v64)
    assert np.array_equal(ids[order], exp_ids)
    assert np.array_equal(lab[order], exp_lab)
    return st


@pytest.mark.parametrize("route", ["sv", "heuristic", "bfs+sv", "sv-theta"])
def test_rmat_hashed_ids(route):
    g = gen.rmat(16, 16, seed=40)
    say(f"[gpu] label64 rmat16 hashed ids route={route}")
    st = check(mix_ids(g.u, 99), mix_ids(g.v, 99), route)
    assert st["sv_passes"] >= 1


def test_duplicate_heavy_and_extreme_ids():
    rng = np.random.default_rng(7)
    pool = np.concatenate([np.asarray([I64_MIN, I64_MAX, -1, 0, 1], np.int64),
                           rng.integers(I64_MIN, I64_MAX, 995, dtype=np.int64)])
    m = 1_000_000
    a = pool[rng.integers(0, 400, m)]                 # 1000 distinct ids at most, 2 M endpoints
    b = pool[rng.integers(0, 400, m)]
    b[::7] = pool[rng.integers(400, 1000, b[::7].shape[0])]
    say("[gpu] label64 duplicate-heavy")
    check(a, b, "sv")
    check(a, b, "heuristic", n_max=1000)              # a tight bound is enough
    # sparse: many components, ids straddling zero
    g = gen.gnm(200_000, 120_000, seed=8)
    check(g.u.astype(np.int64) - 100_000, g.v.astype(np.int64) - 100_000, "sv")


def test_label64_edge_cases():
    z = torch.zeros(0, dtype=torch.int64, device="cuda")
    ids, lab = ccmi.label64(z, z)
    assert ids.numel() == 0 and lab.numel() == 0
    # self-loops only: every id labels itself
    x = np.asarray([5, I64_MIN, 5, I64_MAX], np.int64)
    check(x, x, "sv")
    # a bound below the distinct count is refused
    u = torch.arange(100, dtype=torch.int64, device="cuda")
    with pytest.raises(ccmi.CCError):
        ccmi.label64(u, u + 1, n_max=50)
    # the largest dense case of the test set: C1's G(n,m) with shifted ids
    g = gen.workload("gnm64k")
    check(g.u.astype(np.int64) * 3 + (1 << 50), g.v.astype(np.int64) * 3 + (1 << 50), "heuristic")
