"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import sys

import numpy as np
import torch

import oracle


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_labels_equal(got: torch.Tensor, expect: np.ndarray, what: str):
    g = got.cpu().numpy()
    if not np.array_equal(g, expect):
        bad = np.flatnonzero(g != expect)
        raise AssertionError(f"{what}: {bad.size} labels differ; first at {bad[:5].tolist()}: "
                             f"got {g[bad[:5]].tolist()} expect {expect[bad[:5]].tolist()}")


def oracle_labels(g):
    return oracle.labels_uf(g.u, g.v, g.n)
