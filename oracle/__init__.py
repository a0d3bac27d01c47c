"""ORACLE: plain, slow, obviously correct CPU reference for the connected-components path.

Test infrastructure only.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything under
``oracle/``; the product library never does, and the oracle shares no code with
it (neither imports the other).

What it computes (each function cites the passage it follows):

* ``labels_uf``       -- component labels by sequential union-find (C, ``uf.c``);
                         label = minimum vertex id of the component
                         (Section I definition; Fig. 1(b) caption).
* ``labels_bfs_brute``-- the same labels by one BFS per component in ascending
                         id order (Section I: "a single traversal is necessary for
                         each connected component"); pure Python, tiny graphs.
* ``labels64``        -- arbitrary 64-bit ids: relabel to [0, |V|) in sorted
                         order (Section III-B relabelling; Section V: 64-bit
                         ids), union-find, labels mapped back to original ids.
* ``labels64_brute``  -- the same by BFS over a dict adjacency, seeds in
                         ascending id order; pure Python, tiny graphs.
* ``alg1``            -- the tuple-array algorithm of Section III-A (Algorithm 1)
                         step by step in the paper's notation, small graphs.
* ``degree``          -- degree distribution (Section III-B, Algorithm 2 line
                         "Degree_Distribution"), log-degree bins, histograms.
* ``ks``              -- discrete power-law fit and one-sample K-S statistic
                         (Section III-B; Clauset, Shalizi & Newman 2009).
* ``hybrid``          -- the BFS route of Algorithm 2: seed, visited set,
                         component label, filtered edge list.
* ``mlp``             -- float64 reference of the route-selection MLP.

Every function here is pinned by ``tests/test_oracle*.py`` against things other
than itself: brute force, closed forms, invariants, library routines and the
paper's worked example (``tests/golden/``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import deque

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uf.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile uf.c (gcc -O3; single-threaded by construction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p32 = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_uf_labels.restype = ctypes.c_int64
        lib.oracle_uf_labels.argtypes = [p32, p32, ctypes.c_int64, ctypes.c_int32, p32]
        _lib = lib
    return _lib


def _as_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def labels_uf(u, v, n: int, return_unions: bool = False):
    """Component labels (minimum vertex id per component) by union-find.

    Section I defines components by paths; Fig. 1(b) fixes the label as the
    minimum id.  Raises ValueError if an id is outside [0, n).
    """
    u = _as_i32(u)
    v = _as_i32(v)
    assert u.shape == v.shape
    out = np.empty(max(n, 0), np.int32)
    p32 = ctypes.POINTER(ctypes.c_int32)
    unions = _load().oracle_uf_labels(u.ctypes.data_as(p32), v.ctypes.data_as(p32), u.shape[0], n,
                                      out.ctypes.data_as(p32))
    if unions < 0:
        raise ValueError("vertex id outside [0, n)")
    return (out, int(unions)) if return_unions else out


def labels_bfs_brute(u, v, n: int) -> np.ndarray:
    """One BFS per component, seeds taken in ascending id order, so each
    component is labelled by its smallest vertex (Section I)."""
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    lab = [-1] * n
    for s in range(n):
        if lab[s] != -1:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if lab[y] == -1:
                    lab[y] = s
                    q.append(y)
    return np.asarray(lab, dtype=np.int32)


def component_count(labels: np.ndarray) -> int:
    labels = np.asarray(labels)
    return int(np.count_nonzero(labels == np.arange(labels.shape[0], dtype=labels.dtype)))


def labels64(u, v):
    """Arbitrary 64-bit ids (Section III-B relabels the vertices to [0, |V|);
    Section V: ids are 64-bit integers).  The distinct endpoint ids, sorted,
    become 0 .. n-1, so the relabelling keeps the order and the smallest
    compact id of a component is its smallest original id.  Returns (ids,
    labels): each distinct id once in ascending order, with the smallest id of
    its component."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    ids = np.unique(np.concatenate([u, v]))
    cu = np.searchsorted(ids, u).astype(np.int32)
    cv = np.searchsorted(ids, v).astype(np.int32)
    lab = labels_uf(cu, cv, int(ids.shape[0]))
    return ids, ids[lab]


def labels64_brute(u, v):
    """labels64 by one BFS per component over a dict adjacency, seeds taken
    in ascending id order (Section I)."""
    adj = {}
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        adj.setdefault(a, []).append(b)
        adj.setdefault(b, []).append(a)
    lab = {}
    for s in sorted(adj):
        if s in lab:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if y not in lab:
                    lab[y] = s
                    q.append(y)
    ids = np.asarray(sorted(adj), dtype=np.int64)
    return ids, np.asarray([lab[x] for x in ids.tolist()], dtype=np.int64)
