"""ORACLE (test infrastructure only): the BFS step of Algorithm 2 (Section III-B).

Algorithm 2: compute the degree distribution; if the K-S statistic is below
tau, choose a seed, run a BFS from it to get the visited set VI, remove VI from
V and every edge with an endpoint in VI from E, and then run the SV algorithm
on what is left.

Readings (the paper leaves them open):
* seed: the paper picks a random vertex; here the vertex of maximum degree,
  smallest id on ties (deterministic; it lies in the giant component of a
  scale-free graph with high probability, which is the paper's intent);
* label of the visited component: its minimum vertex id, the same canonical
  label the SV route produces (Fig. 1(b));
* the edge filter drops an edge when its first endpoint is visited (both
  endpoints of an edge share a component, so either test is equivalent).

The visited set is computed by a plain BFS (queue, adjacency lists built with
a stable sort), which tests pin to the component of the seed found by
union-find.
"""
from __future__ import annotations

import numpy as np

from . import degree as _degree


def choose_seed(deg: np.ndarray) -> int:
    """Vertex of maximum degree, smallest id on ties; -1 for an empty graph."""
    deg = np.asarray(deg)
    if deg.shape[0] == 0 or deg.max() <= 0:
        return -1
    return int(np.argmax(deg))          # argmax returns the first maximum


def csr(u, v, n: int):
    """Adjacency lists with both directions of every edge (offsets, targets)."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.argsort(src, kind="stable")
    off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return off, dst[order]


def bfs_visited(u, v, n: int, seed: int) -> np.ndarray:
    """Boolean mask of the vertices reached from seed (level-synchronous BFS)."""
    off, adj = csr(u, v, n)
    vis = np.zeros(n, bool)
    if seed < 0:
        return vis
    vis[seed] = True
    frontier = np.array([seed], np.int64)
    while frontier.shape[0]:
        starts = off[frontier]
        ends = off[frontier + 1]
        lens = ends - starts
        if lens.sum() == 0:
            break
        idx = np.repeat(starts - np.cumsum(np.r_[0, lens[:-1]]), lens) + np.arange(lens.sum())
        nb = adj[idx]
        nb = np.unique(nb[~vis[nb]])
        vis[nb] = True
        frontier = nb
    return vis


def bfs_levels(u, v, n: int, seed: int) -> int:
    """Number of BFS levels (eccentricity of the seed + 1) for reporting."""
    off, adj = csr(u, v, n)
    vis = np.zeros(n, bool)
    if seed < 0:
        return 0
    vis[seed] = True
    frontier = np.array([seed], np.int64)
    levels = 0
    while frontier.shape[0]:
        levels += 1
        starts = off[frontier]
        lens = off[frontier + 1] - starts
        if lens.sum() == 0:
            break
        idx = np.repeat(starts - np.cumsum(np.r_[0, lens[:-1]]), lens) + np.arange(lens.sum())
        nb = adj[idx]
        nb = np.unique(nb[~vis[nb]])
        vis[nb] = True
        frontier = nb
    return levels


def bfs_route(u, v, n: int):
    """Seed, visited mask, component label and the filtered edge list."""
    deg = _degree.degree(u, v, n)
    seed = choose_seed(deg)
    vis = bfs_visited(u, v, n, seed)
    label = int(np.flatnonzero(vis)[0]) if vis.any() else -1
    u = np.asarray(u)
    v = np.asarray(v)
    keep = ~vis[u] if u.shape[0] else np.zeros(0, bool)
    return dict(seed=seed, visited=vis, label=label, u=u[keep], v=v[keep])
