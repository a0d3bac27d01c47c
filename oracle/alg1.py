"""ORACLE (test infrastructure only): the tuple-array algorithm of Section III-A.

This follows Algorithm 1 ("Connected components labeling", Section III-A.2)
in the paper's notation, written from its description:

* the array A holds 3-tuples <p, q, r>; r is a vertex and never changes, p is
  the partition the tuple belongs to, q the candidate partition;
* A_0 has <x, _, x> per vertex x and <x, _, y>, <y, _, x> per edge {x, y};
* an iteration groups A by r (vertex buckets VB(u)), writes the nominated
  partition u_min = min M(u) into q; then groups A by p (partition buckets
  PB(p)), lets each partition join p_min = min C(p) and records a temporary
  tuple <p_min, _, p_min>; the two groupings are then repeated once with the
  temporary tuples present (pointer doubling, Fig. "doubling"), and the
  temporary tuples are erased;
* the loop stops when every partition satisfies p = p_min;
* the label of u is the first element of any tuple <c, _, u>.

Grouping uses a stable sort (the paper sorts; here one process holds all of
A).  The optional ``exclude_completed`` implements Section III-A.4: a tuple is
"potentially completed" when its vertex bucket has a single partition, and a
partition whose tuples are all potentially completed is set aside.

Small graphs only (pure numpy, O(log n) sorts of O(n + m) tuples).
"""
from __future__ import annotations

import numpy as np

NONE = np.iinfo(np.int64).max   # the "_" placeholder


def initial_tuples(u, v, n: int):
    """A_0 (Algorithm 1, initialisation): one tuple per vertex, two per edge."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    x = np.arange(n, dtype=np.int64)
    p = np.concatenate([x, u, v])
    r = np.concatenate([x, v, u])
    q = np.full(p.shape, NONE, np.int64)
    return p, q, r


# ---------------------------------------------------------------- notation
def partitions(p):
    """P_i: the distinct first entries."""
    return set(np.unique(p).tolist())


def partition_bucket(p, q, r, part):
    """PB_i(part): tuples whose first entry is part."""
    sel = p == part
    return list(zip(p[sel].tolist(), q[sel].tolist(), r[sel].tolist()))


def vertex_bucket(p, q, r, u):
    """VB_i(u): tuples whose third entry is u."""
    sel = r == u
    return list(zip(p[sel].tolist(), q[sel].tolist(), r[sel].tolist()))


def vertex_members(p, r, part):
    """V_i(part) = {r : <part, q, r> in PB_i(part)}."""
    return set(r[p == part].tolist())


def candidates(p, q, part):
    """C_i(part) = {q : <part, q, r> in PB_i(part)}."""
    return set(q[p == part].tolist())


def partitions_of_vertex(p, r, u):
    """M_i(u) = {p : <p, q, u> in VB_i(u)}."""
    return set(p[r == u].tolist())


def neighborhood(p, r, part):
    """N_i(part) = union of M_i(u) over u in V_i(part)."""
    out = set()
    for u in vertex_members(p, r, part):
        out |= partitions_of_vertex(p, r, u)
    return out


# ------------------------------------------------------------------ steps
def _group_min(keys, vals):
    """Sort by key, then the minimum of vals over each run of equal keys,
    broadcast back to every tuple of the run (the bucket scan after a sort)."""
    if keys.shape[0] == 0:
        return vals.copy()
    order = np.argsort(keys, kind="stable")
    ks = keys[order]
    vs = vals[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    mins = np.minimum.reduceat(vs, starts)
    run_id = np.cumsum(np.r_[False, ks[1:] != ks[:-1]])
    out = np.empty_like(vals)
    out[order] = mins[run_id]
    return out


def nominate(p, q, r):
    """Group by r: every tuple of VB(u) gets q <- u_min = min M(u)."""
    return _group_min(r, p)


def join_min_candidate(p, q):
    """Group by p: every tuple of PB(p) gets p <- p_min = min C(p).
    Returns the new first entries and whether some partition changed."""
    pmin = _group_min(p, q)
    return pmin, bool(np.any(pmin != p))


def run(u, v, n: int, exclude_completed: bool = False, max_iter: int = 10_000):
    """Algorithm 1 until convergence.  Returns (labels, iterations)."""
    p, q, r = initial_tuples(u, v, n)
    done_p = np.empty(0, np.int64)
    done_r = np.empty(0, np.int64)
    it = 0
    converged = False
    while not converged:
        it += 1
        if it > max_iter:
            raise RuntimeError("Algorithm 1 did not converge")
        converged = True
        # first pair of groupings: p joins min N(p)
        q = nominate(p, q, r)
        if exclude_completed:
            # |M(u)| = 1  <=>  min and max partition of the vertex bucket agree
            maxp = -_group_min(r, -p)
            pot = maxp == q
        newp, changed = join_min_candidate(p, q)
        if changed:
            converged = False
        if exclude_completed:
            # partition completed iff all of its tuples are potentially completed
            allpot = _group_min(p, pot.astype(np.int64)) == 1
            done = allpot & (newp == p)
            if np.any(done):
                done_p = np.concatenate([done_p, p[done]])
                done_r = np.concatenate([done_r, r[done]])
                keep = ~done
                p, q, r, newp = p[keep], q[keep], r[keep], newp[keep]
        # temporary tuples <p_min, _, p_min>, one per partition of this iteration
        tmp = np.unique(newp)
        p = np.concatenate([newp, tmp])
        q = np.concatenate([q, np.full(tmp.shape, NONE, np.int64)])
        r = np.concatenate([r, tmp])
        is_tmp = np.r_[np.zeros(newp.shape[0], bool), np.ones(tmp.shape[0], bool)]
        # second pair of groupings: p_min joins min M(p_min) (pointer doubling)
        q = nominate(p, q, r)
        p2, changed2 = join_min_candidate(p, q)
        if changed2:
            converged = False
        # erase the temporary tuples
        p, q, r = p2[~is_tmp], q[~is_tmp], r[~is_tmp]
    labels = np.empty(n, np.int64)
    labels[r] = p
    if done_r.shape[0]:
        labels[done_r] = done_p
    return labels.astype(np.int32), it
