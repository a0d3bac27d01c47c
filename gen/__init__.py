"""Seeded synthetic graph inputs (shared by the tests, the benchmark and the oracle checks).

This module only draws random graphs; it holds none of the connected-components
arithmetic.  The C generators in ``gen.c`` are counter-based, so each output is a
pure function of the seed.  Workload recipes (sizes, seeds, value distributions)
mirror the paper's graph families (Section IV, Table "tab:data"); the real
datasets are not available, and these synthetic inputs stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile gen.c into libgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.gen_gnm.restype = ctypes.c_int64
        lib.gen_gnm.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, I32P, I32P]
        lib.gen_rmat.restype = None
        lib.gen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                 I32P, I32P]
        lib.gen_grid.restype = ctypes.c_int64
        lib.gen_grid.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int, I32P, I32P]
        lib.gen_plcomp.restype = ctypes.c_int64
        lib.gen_plcomp.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                   I32P, I32P, ctypes.c_int64]
        lib.gen_plcomp_sizes.restype = ctypes.c_int64
        lib.gen_plcomp_sizes.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_uint64, I32P, ctypes.c_int64]
        lib.gen_permutation.restype = None
        lib.gen_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, I32P]
        lib.gen_shuffle_edges.restype = None
        lib.gen_shuffle_edges.argtypes = [ctypes.c_int64, ctypes.c_uint64, I32P, I32P]
        lib.gen_batch_plan.restype = ctypes.c_int
        lib.gen_batch_plan.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       I32P, I64P, I32P]
        lib.gen_batch_fetch.restype = ctypes.c_int
        lib.gen_batch_fetch.argtypes = [I32P, I32P]
        lib.gen_batch_discard.restype = None
        lib.gen_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(I32P)


def _p64(a: np.ndarray):
    return a.ctypes.data_as(I64P)


@dataclass
class Graph:
    """An undirected edge list: edge i joins u[i] and v[i]; ids lie in [0, n)."""
    u: np.ndarray
    v: np.ndarray
    n: int
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])


def gnm(n: int, m: int, seed: int) -> Graph:
    """G(n,m): m distinct unordered pairs drawn uniformly, no self-loops."""
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    k = _load().gen_gnm(n, m, seed, _p32(u), _p32(v))
    if k < 0:
        raise MemoryError("gen_gnm")
    return Graph(u[:k].copy() if k < m else u, v[:k].copy() if k < m else v, n, f"gnm(n={n},m={m},seed={seed})")


def rmat(scale: int, edge_factor: float, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, permute: bool = True, m: int | None = None, noise: float = 0.0) -> Graph:
    """R-MAT: 2^scale vertices, edge_factor * 2^scale edges, one quadrant draw per
    level; noise > 0 perturbs the quadrant probabilities per level (noisy SKG)."""
    n = 1 << scale
    if m is None:
        m = int(round(edge_factor * n))
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    _load().gen_rmat(scale, m, a, b, c, noise, seed, 1 if permute else 0, _p32(u), _p32(v))
    return Graph(u, v, n, f"rmat(scale={scale},ef={edge_factor},seed={seed},noise={noise})")


def grid(L: int, p: float, seed: int, permute: bool = True, shuffle: bool = True) -> Graph:
    """L x L lattice with each of the 2L(L-1) edges kept with probability p."""
    cap = 2 * L * (L - 1)
    u = np.empty(max(cap, 1), np.int32)
    v = np.empty(max(cap, 1), np.int32)
    m = _load().gen_grid(L, p, seed, 1 if permute else 0, 1 if shuffle else 0, _p32(u), _p32(v))
    if m < cap:
        u = u[:m].copy()
        v = v[:m].copy()
    return Graph(u, v, L * L, f"grid(L={L},p={p},seed={seed})")


PL_LAMBDA = 3.5   # chords per vertex drawn before the degree-cap and duplicate skips (gives ~1.25 edges/vertex)
PL_WINDOW = 16
PL_MAXDEG = 8


def plcomp(n: int, seed: int, expo: float = 2.5, smax: int = 100_000, lam: float = PL_LAMBDA,
           window: int = PL_WINDOW, maxdeg: int = PL_MAXDEG, permute: bool = True) -> Graph:
    """Forest of power-law-sized components, each a path with branches and chords."""
    smax = min(smax, n)
    cap = 5 * n + 16
    u = np.empty(cap, np.int32)
    v = np.empty(cap, np.int32)
    m = _load().gen_plcomp(n, expo, smax, lam, window, maxdeg, seed, 1 if permute else 0,
                           _p32(u), _p32(v), cap)
    if m < 0:
        raise MemoryError("gen_plcomp")
    return Graph(u[:m].copy(), v[:m].copy(), n, f"plcomp(n={n},seed={seed})")


def plcomp_sizes(n: int, seed: int, expo: float = 2.5, smax: int = 100_000) -> np.ndarray:
    smax = min(smax, n)
    out = np.empty(n + 1, np.int32)
    c = _load().gen_plcomp_sizes(n, expo, smax, seed, _p32(out), n + 1)
    return out[:c].copy()


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    _load().gen_permutation(n, seed, _p32(out))
    return out


@dataclass
class Batch:
    """G graphs with graph-local ids, concatenated; graph g owns edges
    [edge_off[g], edge_off[g+1]) and vertices [vert_off[g], vert_off[g+1])."""
    u: np.ndarray
    v: np.ndarray
    edge_off: np.ndarray
    vert_off: np.ndarray
    family: np.ndarray

    @property
    def G(self) -> int:
        return int(self.edge_off.shape[0] - 1)

    def graph(self, g: int) -> Graph:
        a, b = int(self.edge_off[g]), int(self.edge_off[g + 1])
        n = int(self.vert_off[g + 1] - self.vert_off[g])
        return Graph(self.u[a:b], self.v[a:b], n, f"batch[{g}]")


def batch(G: int, seed_base: int, lg_lo: float = 8.0, lg_hi: float = 20.0,
          d_lo: float = 2.0, d_hi: float = 16.0) -> Batch:
    lib = _load()
    n = np.empty(G, np.int32)
    m = np.empty(G, np.int64)
    fam = np.empty(G, np.int32)
    rc = lib.gen_batch_plan(G, seed_base, lg_lo, lg_hi, d_lo, d_hi, _p32(n), _p64(m), _p32(fam))
    if rc != 0:
        lib.gen_batch_discard()
        raise RuntimeError(f"gen_batch_plan failed ({rc})")
    edge_off = np.zeros(G + 1, np.int64)
    edge_off[1:] = np.cumsum(m)
    vert_off = np.zeros(G + 1, np.int64)
    vert_off[1:] = np.cumsum(n.astype(np.int64))
    tot = int(edge_off[-1])
    u = np.empty(max(tot, 1), np.int32)
    v = np.empty(max(tot, 1), np.int32)
    lib.gen_batch_fetch(_p32(u), _p32(v))
    return Batch(u[:tot], v[:tot], edge_off, vert_off, fam)


# --------------------------------------------------------------- workloads
# The five workloads: (1) G(n,m) near-critical, (2) R-MAT scale 24 / edge factor
# 16, (3) 8192^2 lattice thinned at p = 0.7, (4) 200 M-vertex power-law
# component forest, (5) a batch of 4096 uneven graphs.  Each has a small
# variant (same recipe, smaller size) that the oracle finishes in seconds.

def workload(name: str):
    if name == "gnm64k":
        return gnm(65536, 65536, seed=1)
    if name == "rmat24":
        return rmat(24, 16, seed=2)
    if name == "grid8192":
        return grid(8192, 0.7, seed=3)
    if name == "plcomp200m":
        return plcomp(200_000_000, seed=4)
    if name == "batch4096":
        return batch(4096, 5_000_000)
    # small variants
    if name == "rmat16":
        return rmat(16, 16, seed=2)
    if name == "rmat18":
        return rmat(18, 16, seed=2)
    if name == "rmat18noisy":
        return rmat(18, 16, seed=2, noise=0.1)
    if name == "rmat24noisy":
        return rmat(24, 16, seed=2, noise=0.1)
    if name == "grid512":
        return grid(512, 0.7, seed=3)
    if name == "plcomp1m":
        return plcomp(1_000_000, seed=4)
    if name == "batch64":
        return batch(64, 5_000_000, lg_hi=14.0)
    raise KeyError(name)


WORKLOADS_FULL = ["gnm64k", "rmat24", "grid8192", "plcomp200m", "batch4096"]
