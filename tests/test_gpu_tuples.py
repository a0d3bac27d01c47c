"""GPU parity of cc_label_tuples (Algorithm 1 with radix sorts) against the
oracle: labels bit-exact against union-find, and the number of iterations
equal to the oracle's step-by-step transcription of Algorithm 1 (the same
tuples are formed in the same order of steps, so the loop must stop at the
same iteration)."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import assert_labels_equal, oracle_labels, say, to_dev
from oracle import alg1

pytestmark = pytest.mark.gpu
ccmi = pytest.importorskip("paper_1607_06156_amd")


def run(g, exclude=False):
    say(f"[gpu] tuples {g.name} n={g.n} m={g.m} exclude={exclude}")
    lab, st = ccmi.label_tuples(to_dev(g.u), to_dev(g.v), g.n, exclude=exclude)
    say(f"   iterations={st['iterations']} sorts={st['sorts']} passes={st['passes_per_sort']} "
        f"sort {st['ms_sort']:.2f} of {st['ms_total']:.2f} ms")
    return lab, st


@pytest.mark.parametrize("name,g", [
    ("gnm", gen.gnm(3000, 2500, seed=1)),
    ("rmat", gen.rmat(11, 4, seed=2)),
    ("grid", gen.grid(40, 0.6, seed=3)),
    ("plcomp", gen.plcomp(20_000, seed=4)),
    ("gnm-dense", gen.gnm(500, 4000, seed=5)),
])
def test_tuples_match_algorithm1_oracle(name, g):
    lab, st = run(g)
    exp, it = alg1.run(g.u, g.v, g.n)
    assert_labels_equal(lab, exp, name)
    assert_labels_equal(lab, oracle_labels(g), name)
    assert st["iterations"] == it
    assert st["sorts"] == 4 * it and st["tuples"] == g.n + 2 * g.m


@pytest.mark.parametrize("name,g", [
    ("gnm", gen.gnm(3000, 2500, seed=1)),
    ("rmat", gen.rmat(11, 4, seed=2)),
    ("grid", gen.grid(40, 0.6, seed=3)),
    ("plcomp", gen.plcomp(20_000, seed=4)),
])
def test_tuples_with_exclusion_match_oracle(name, g):
    """Completed partitions set aside (Section III-A.4): same labels, and the
    iteration count of the oracle transcription run with the same option."""
    lab, st = run(g, exclude=True)
    exp, it = alg1.run(g.u, g.v, g.n, exclude_completed=True)
    assert_labels_equal(lab, exp, name)
    assert_labels_equal(lab, oracle_labels(g), name)
    assert st["iterations"] == it


def test_tuples_closed_forms_and_ragged_sizes():
    rng = np.random.default_rng(3)
    n = 5000
    perm = rng.permutation(n).astype(np.int32)
    path = gen.Graph(perm[:-1], perm[1:], n, "path")                   # one component
    lab, _ = run(path)
    assert_labels_equal(lab, np.zeros(n, np.int32), "path")
    none = gen.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), 77, "no edges")
    lab, st = run(none)
    assert_labels_equal(lab, np.arange(77, dtype=np.int32), "no edges")
    loops = gen.Graph(np.arange(9, dtype=np.int32), np.arange(9, dtype=np.int32), 9, "self-loops")
    lab, _ = run(loops)
    assert_labels_equal(lab, np.arange(9, dtype=np.int32), "self-loops")
    for m in [1, 5, 1023, 4095, 4097, 70001]:                         # around the 4096-tuple tile
        g = gen.gnm(max(8, m), m, seed=m)
        for ex in (False, True):
            lab, _ = run(g, exclude=ex)
            assert_labels_equal(lab, oracle_labels(g), f"gnm m={m} exclude={ex}")
    lab, _ = run(loops, exclude=True)                                  # every partition completes at once
    assert_labels_equal(lab, np.arange(9, dtype=np.int32), "self-loops, exclusion")


def test_tuples_medium_graphs():
    for g in (gen.workload("rmat16"), gen.workload("grid512"), gen.workload("gnm64k")):
        lab, st = run(g)
        assert_labels_equal(lab, oracle_labels(g), g.name)
        assert 0 < st["ms_sort"] <= st["ms_total"]


def test_tuples_range_error():
    u = to_dev(np.asarray([0, 5], np.int32))
    v = to_dev(np.asarray([1, 2], np.int32))
    with pytest.raises(ccmi.CCError):
        ccmi.label_tuples(u, v, 4)
