"""ORACLE (test infrastructure only): power-law fit and K-S statistic of the degree distribution.

Section III-B classifies a graph as scale-free when its degree distribution
fits a power law: the fit follows Clauset, Shalizi & Newman (SIAM Review 2009)
for discrete data and the goodness of fit is the one-sample
Kolmogorov-Smirnov statistic; BFS runs first iff the statistic is below a
user threshold tau, set to 0.05 in Section V ("Hybrid Implementation
Analysis", Table "tab:ks_stat").

Model, for a lower cutoff d_min:  P(d) = d^-alpha / zeta(alpha, d_min), d >= d_min,
with the Hurwitz zeta function zeta(s, q) = sum_{k>=0} (q + k)^-s.
Steps, in the order Clauset et al. give them:
 1. for each candidate d_min, estimate alpha by maximum likelihood: the
    log-likelihood is  -alpha * sum(ln d_i) - N ln zeta(alpha, d_min), whose
    stationary point solves  E_alpha[ln d] = mean(ln d_i);  E_alpha[ln d] falls
    monotonically in alpha, so bisection on (1, 10] finds it;
 2. D(d_min) = max over integers d in [d_min, d_max] of |S(d) - P(D <= d)|,
    S the empirical CDF of the tail and P(D <= d) = 1 - zeta(alpha, d+1)/zeta(alpha, d_min);
    between consecutive observed degrees S is flat and the model CDF rises, so
    the maximum is attained at an observed degree or just before the next one;
 3. d_min is the candidate with the smallest D; the statistic is that D.

Readings where the paper is silent (it uses the plfit library): degree 0 is
excluded; candidates are the distinct degrees whose tail holds at least 50
vertices and at least 2 distinct values; alpha is searched on (1, 10]; ties in
D pick the smaller d_min.

The Hurwitz zeta function and its derivative in s are evaluated by the
Euler-Maclaurin formula (N = 12 direct terms, 7 Bernoulli corrections), which
tests pin against scipy.special.zeta.
"""
from __future__ import annotations

import math

import numpy as np

MIN_TAIL = 50
ALPHA_LO = 1.0 + 1e-9
ALPHA_HI = 10.0
TAU = 0.05

# B_{2j} / (2j)! for j = 1..7
_B2J = [1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730, 7.0 / 6]
_C2J = [b / math.factorial(2 * (j + 1)) for j, b in enumerate(_B2J)]
_NDIRECT = 12


def hurwitz_zeta(s, q):
    """zeta(s, q) for s > 1, q >= 1 (vectorised, float64), Euler-Maclaurin."""
    s = np.asarray(s, np.float64)
    q = np.asarray(q, np.float64)
    s, q = np.broadcast_arrays(s, q)
    acc = np.zeros(s.shape)
    for k in range(_NDIRECT):
        acc += (q + k) ** (-s)
    a = q + _NDIRECT
    acc += a ** (1.0 - s) / (s - 1.0) + 0.5 * a ** (-s)
    rising = s.copy()                 # (s)_{2j-1} for j = 1
    for j, c in enumerate(_C2J):
        jj = j + 1
        acc += c * rising * a ** (-s - 2 * jj + 1)
        rising = rising * (s + 2 * jj - 1) * (s + 2 * jj)
    return acc


def hurwitz_zeta_ds(s, q):
    """d/ds zeta(s, q), term by term from the same expansion."""
    s = np.asarray(s, np.float64)
    q = np.asarray(q, np.float64)
    s, q = np.broadcast_arrays(s, q)
    acc = np.zeros(s.shape)
    for k in range(_NDIRECT):
        acc -= np.log(q + k) * (q + k) ** (-s)
    a = q + _NDIRECT
    la = np.log(a)
    acc -= a ** (1.0 - s) * (la / (s - 1.0) + 1.0 / (s - 1.0) ** 2)
    acc -= 0.5 * la * a ** (-s)
    rising = s.copy()
    drising = np.ones(s.shape)        # derivative of (s)_{2j-1}
    for j, c in enumerate(_C2J):
        jj = j + 1
        p = a ** (-s - 2 * jj + 1)
        acc += c * (drising - rising * la) * p
        f1 = s + 2 * jj - 1
        f2 = s + 2 * jj
        drising = drising * f1 * f2 + rising * (f1 + f2)
        rising = rising * f1 * f2
    return acc


def mle_alpha(dmin, mean_log, iters: int = 200):
    """Solve E_alpha[ln d | d >= dmin] = mean_log by bisection (vectorised)."""
    dmin = np.asarray(dmin, np.float64)
    mean_log = np.asarray(mean_log, np.float64)
    lo = np.full(dmin.shape, ALPHA_LO)
    hi = np.full(dmin.shape, ALPHA_HI)

    def f(a):
        return -hurwitz_zeta_ds(a, dmin) / hurwitz_zeta(a, dmin) - mean_log

    at_hi = f(hi) >= 0          # still above the target at the upper bound: clamp
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = f(mid) > 0        # E[ln d] too large -> alpha must grow
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
        if np.all(hi - lo <= 1e-15 * hi):
            break
    return np.where(at_hi, ALPHA_HI, 0.5 * (lo + hi))


def ks_distance(vals: np.ndarray, cnts: np.ndarray, dmin: int, alpha: float, observed_only: bool = False) -> float:
    """D(dmin) for a given alpha; vals sorted ascending, all >= dmin.

    observed_only: the other reading of step 2, with the gap taken only at
    the observed degrees d_j (not on the integers in between)."""
    N = float(cnts.sum())
    S = np.cumsum(cnts) / N                       # S(d_j)
    z0 = hurwitz_zeta(alpha, float(dmin))
    F_at = 1.0 - hurwitz_zeta(alpha, vals + 1.0) / z0          # model CDF at d_j
    dev = np.abs(S - F_at)
    if observed_only:
        return float(np.max(dev))
    if vals.shape[0] > 1:
        # just before the next observed value: S still S(d_j), model at d_{j+1} - 1
        F_before = 1.0 - hurwitz_zeta(alpha, vals[1:].astype(np.float64)) / z0
        dev = np.maximum(dev[:-1], np.abs(S[:-1] - F_before)).tolist() + [dev[-1]]
        return float(np.max(dev))
    return float(np.max(dev))


def fit(vals, cnts, observed_only: bool = False):
    """Clauset fit over all candidate cutoffs.

    vals: distinct positive degrees (any order); cnts: vertices per degree.
    Returns dict(ks, alpha, dmin, ntail, candidates).  ks = inf when no
    candidate cutoff exists (the graph is then never classed scale-free).
    observed_only selects the reading of step 2 that takes the gap at the
    observed degrees only (see ks_distance).
    """
    vals = np.asarray(vals, np.int64)
    cnts = np.asarray(cnts, np.int64)
    keep = vals > 0
    vals, cnts = vals[keep], cnts[keep]
    order = np.argsort(vals)
    vals, cnts = vals[order], cnts[order]
    if vals.shape[0] < 2:
        return dict(ks=math.inf, alpha=math.nan, dmin=0, ntail=0, candidates=0)
    logs = np.log(vals.astype(np.float64))
    # suffix sums over the sorted distinct values
    tail_n = np.cumsum(cnts[::-1])[::-1]
    tail_s = np.cumsum((cnts * logs)[::-1])[::-1]
    ndist = vals.shape[0] - np.arange(vals.shape[0])
    cand = np.flatnonzero((tail_n >= MIN_TAIL) & (ndist >= 2))
    if cand.shape[0] == 0:
        return dict(ks=math.inf, alpha=math.nan, dmin=0, ntail=0, candidates=0)
    alphas = mle_alpha(vals[cand], tail_s[cand] / tail_n[cand])
    best = None
    for i, a in zip(cand.tolist(), alphas.tolist()):
        D = ks_distance(vals[i:], cnts[i:], int(vals[i]), a, observed_only)
        if best is None or D < best[0]:
            best = (D, a, int(vals[i]), int(tail_n[i]))
    return dict(ks=best[0], alpha=best[1], dmin=best[2], ntail=best[3], candidates=int(cand.shape[0]))


def decide_bfs(ks_value: float, tau: float = TAU) -> bool:
    """Algorithm 2: run the BFS step iff the statistic is strictly below tau."""
    return bool(ks_value < tau)
