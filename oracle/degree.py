"""ORACLE (test infrastructure only): degree distribution and histograms.

Section III-B (Algorithm 2, first step) computes the degree distribution D of
the graph; each undirected edge is stored as two directed edges, so a vertex's
degree is the number of edge endpoints equal to it and a self-loop adds 2.

Histograms used by the route decision:
* ``exact``  -- counts of vertices with degree d for 0 <= d < 4096;
* ``tail``   -- the individual degrees >= 4096 (one entry per vertex);
* ``log64``  -- 64 half-octave bins: bin 0 holds degree 0; a degree d >= 1 with
                k = floor(log2 d) goes to 1 + 2k, plus 1 when k >= 1 and the bit
                just below the leading one is set.  (Bin layout is this
                library's choice; the paper fixes only D itself.)
"""
from __future__ import annotations

import numpy as np

EXACT_BINS = 4096


def degree(u, v, n: int) -> np.ndarray:
    """deg[x] = number of edge endpoints equal to x (directed doubling)."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    return (np.bincount(u, minlength=n) + np.bincount(v, minlength=n)).astype(np.int64)


def log_bin(d: int) -> int:
    """Half-octave bin of one degree, written out with plain integer steps."""
    if d == 0:
        return 0
    k = d.bit_length() - 1
    extra = (d >> (k - 1)) & 1 if k >= 1 else 0
    return 1 + 2 * k + extra


def log_bins(deg: np.ndarray) -> np.ndarray:
    deg = np.asarray(deg, np.int64)
    out = np.zeros(deg.shape, np.int64)
    pos = deg > 0
    d = deg[pos]
    k = np.floor(np.log2(d.astype(np.float64))).astype(np.int64)
    # guard float rounding of log2 near powers of two
    k = np.where((np.int64(1) << (k + 1)) <= d, k + 1, k)
    k = np.where((np.int64(1) << k) > d, k - 1, k)
    extra = np.where(k >= 1, (d >> np.maximum(k - 1, 0)) & 1, 0)
    out[pos] = 1 + 2 * k + extra
    return out


def histograms(deg: np.ndarray):
    """(log64[64], exact[4096], sorted tail degrees) as int64 arrays."""
    deg = np.asarray(deg, np.int64)
    log64 = np.bincount(log_bins(deg), minlength=64).astype(np.int64)
    small = deg[deg < EXACT_BINS]
    exact = np.bincount(small, minlength=EXACT_BINS).astype(np.int64)
    tail = np.sort(deg[deg >= EXACT_BINS])
    return log64, exact, tail


def distribution(deg: np.ndarray):
    """Degree distribution D as (distinct positive degrees, vertex counts)."""
    deg = np.asarray(deg, np.int64)
    vals, cnts = np.unique(deg[deg > 0], return_counts=True)
    return vals, cnts.astype(np.int64)


def distribution_from_histograms(exact: np.ndarray, tail: np.ndarray):
    vals = np.flatnonzero(exact)
    vals = vals[vals > 0]
    cnts = exact[vals]
    tv, tc = np.unique(np.asarray(tail, np.int64), return_counts=True)
    return np.concatenate([vals.astype(np.int64), tv]), np.concatenate([cnts.astype(np.int64), tc])


def router_features(log64: np.ndarray, n: int, m: int) -> np.ndarray:
    """66 features: log-degree histogram / n, log2 n, log2 m (log2 of max(., 1))."""
    f = np.zeros(66, np.float64)
    f[:64] = np.asarray(log64, np.float64) / max(n, 1)
    f[64] = np.log2(max(n, 1))
    f[65] = np.log2(max(m, 1))
    return f
