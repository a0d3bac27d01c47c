"""Pins for the degree / histogram / power-law-fit oracles."""
import math

import numpy as np
import pytest
import scipy.special as ss

import gen
from oracle import degree as odeg
from oracle import ks


# ------------------------------------------------------------------ degree
def test_degree_counts_endpoints_selfloop_twice():
    u = [0, 1, 2, 2, 3]
    v = [1, 2, 2, 0, 3]
    # brute force: count endpoint occurrences
    exp = [0] * 5
    for a, b in zip(u, v):
        exp[a] += 1
        exp[b] += 1
    assert odeg.degree(u, v, 5).tolist() == exp == [2, 2, 4, 2, 0]


def test_degree_handshake_and_regular_graphs():
    g = gen.rmat(14, 8, seed=1)
    d = odeg.degree(g.u, g.v, g.n)
    assert d.sum() == 2 * g.m                       # handshake lemma
    # complete grid: corner 2, border 3, interior 4
    L = 20
    gg = gen.grid(L, 1.0, seed=0, permute=False, shuffle=False)
    dd = odeg.degree(gg.u, gg.v, gg.n).reshape(L, L)
    assert dd[0, 0] == 2 and dd[0, 5] == 3 and dd[5, 5] == 4


def test_log_bin_definition():
    assert odeg.log_bin(0) == 0 and odeg.log_bin(1) == 1
    for k in range(1, 31):
        assert odeg.log_bin(1 << k) == 1 + 2 * k
        assert odeg.log_bin(3 << (k - 1)) == 2 + 2 * k
        assert odeg.log_bin((1 << (k + 1)) - 1) == 2 + 2 * k
    assert odeg.log_bin(2 ** 31 - 1) == 62
    d = np.concatenate([np.arange(0, 1 << 16), np.random.default_rng(0).integers(0, 2 ** 31 - 1, 20000)])
    assert np.array_equal(odeg.log_bins(d), np.array([odeg.log_bin(int(x)) for x in d]))
    b = odeg.log_bins(np.arange(0, 1 << 16))
    assert np.all(np.diff(b) >= 0)                   # monotone in d


def test_histograms_partition_vertices():
    g = gen.rmat(16, 16, seed=2)
    d = odeg.degree(g.u, g.v, g.n)
    log64, exact, tail = odeg.histograms(d)
    assert log64.sum() == g.n
    assert exact.sum() + tail.shape[0] == g.n
    vals, cnts = odeg.distribution(d)
    v2, c2 = odeg.distribution_from_histograms(exact, tail)
    o = np.argsort(v2)
    assert np.array_equal(vals, v2[o]) and np.array_equal(cnts, c2[o])


# ------------------------------------------------------------ Hurwitz zeta
def test_zeta_closed_forms():
    assert abs(ks.hurwitz_zeta(2.0, 1.0) - math.pi ** 2 / 6) < 1e-14
    assert abs(ks.hurwitz_zeta(4.0, 1.0) - math.pi ** 4 / 90) < 1e-14
    # recurrence zeta(s, q) - zeta(s, q + 1) = q^-s
    for s in [1.1, 2.5, 7.0]:
        for q in [1.0, 3.0, 17.0, 1000.0]:
            lhs = ks.hurwitz_zeta(s, q) - ks.hurwitz_zeta(s, q + 1)
            # the difference cancels: allow a few ulps of zeta(s, q) itself
            assert abs(lhs - q ** -s) <= 2e-15 * ks.hurwitz_zeta(s, q)


def test_zeta_vs_scipy():
    s = np.linspace(1.01, 10.0, 60)
    for q in [1.0, 2.0, 5.0, 50.0, 4096.0, 1e6]:
        ref = ss.zeta(s, q)
        got = ks.hurwitz_zeta(s, q)
        assert np.max(np.abs(got / ref - 1)) < 1e-12


def test_zeta_derivative_vs_finite_differences():
    for s in [1.05, 1.5, 2.2, 3.7, 8.0]:
        for q in [1.0, 6.0, 300.0]:
            h = 1e-5 * s
            fd = (ss.zeta(s + h, q) - ss.zeta(s - h, q)) / (2 * h)
            got = float(ks.hurwitz_zeta_ds(s, q))
            assert abs(got / fd - 1) < 1e-7, (s, q)


# ------------------------------------------------------------- power law fit
def _exact_powerlaw_counts(alpha, dmin, dmax, N=1e15):
    d = np.arange(dmin, dmax + 1)
    pmf = d.astype(float) ** -alpha / ss.zeta(alpha, dmin)
    return d, np.round(N * pmf).astype(np.int64)


@pytest.mark.parametrize("alpha", [2.8, 3.5])
def test_fit_recovers_exact_power_law(alpha):
    """Counts proportional to the model pmf (steep enough that the mass beyond
    d = 1500 is below 1e-6): the fit returns the generating alpha and D ~ 0."""
    d, c = _exact_powerlaw_counts(alpha, 1, 1500)
    r = ks.fit(d, c)
    assert r["dmin"] == 1
    assert abs(r["alpha"] - alpha) < 1e-3
    assert r["ks"] < 1e-5


@pytest.mark.parametrize("alpha", [1.5, 2.2, 3.0, 6.0])
@pytest.mark.parametrize("dmin", [1, 5, 40])
def test_mle_solves_score_equation(alpha, dmin):
    """The untruncated model's mean log-degree, -d/ds ln zeta(s, dmin) at s = alpha
    (finite differences of scipy's zeta), must give back alpha."""
    h = 1e-5
    mean_log = -(np.log(ss.zeta(alpha + h, dmin)) - np.log(ss.zeta(alpha - h, dmin))) / (2 * h)
    got = float(ks.mle_alpha(np.array([float(dmin)]), np.array([mean_log]))[0])
    assert abs(got - alpha) < 1e-6 * alpha


def test_ks_distance_vs_full_enumeration():
    """D from the jump points equals the maximum over every integer in range."""
    rng = np.random.default_rng(9)
    for trial in range(20):
        vals = np.unique(rng.integers(3, 400, int(rng.integers(2, 60))))
        cnts = rng.integers(1, 1000, vals.shape[0])
        alpha = float(rng.uniform(1.3, 4.0))
        dmin = int(vals[0])
        got = ks.ks_distance(vals, cnts, dmin, alpha)
        allv = np.arange(dmin, vals[-1] + 1)
        S = np.array([cnts[vals <= x].sum() for x in allv]) / cnts.sum()
        F = 1.0 - ss.zeta(alpha, allv + 1.0) / ss.zeta(alpha, dmin)
        assert abs(got - np.max(np.abs(S - F))) < 1e-12


def test_fit_finds_the_cutoff():
    """Counts below d0 do not follow the law; above they do: d_min = d0, D ~ 0."""
    d0 = 12
    d, c = _exact_powerlaw_counts(4.0, d0, 1500)
    low = np.arange(1, d0)
    lowc = np.full(low.shape, int(c[0] * 3))
    r = ks.fit(np.concatenate([low, d]), np.concatenate([lowc, c]))
    assert r["dmin"] == d0
    assert abs(r["alpha"] - 4.0) < 1e-3
    assert r["ks"] < 1e-5


def test_clauset_approximation_agrees():
    """alpha ~ 1 + N / sum(ln(d_i / (dmin - 1/2))) (Clauset et al. eq. 3.7) within 2 % for dmin >= 6."""
    rng = np.random.default_rng(4)
    alpha, dmin = 2.6, 8
    d = np.arange(dmin, 2_000_000)
    pmf = d.astype(float) ** -alpha
    cdf = np.cumsum(pmf) / pmf.sum()
    x = d[np.searchsorted(cdf, rng.random(200_000))]
    vals, cnts = np.unique(x, return_counts=True)
    a_mle = float(ks.mle_alpha(np.array([float(dmin)]), np.array([np.log(x).mean()]))[0])
    a_approx = 1 + x.shape[0] / np.sum(np.log(x / (dmin - 0.5)))
    assert abs(a_mle / a_approx - 1) < 0.02
    assert abs(a_mle - alpha) < 0.05


def test_statistic_separates_families():
    """Power-law-like degree sequences fall below tau = 0.05, Poisson and lattice
    degrees do not (the separation pattern of Table "tab:ks_stat")."""
    rng = np.random.default_rng(6)
    d = np.arange(1, 5_000_000)
    cdf = np.cumsum(d.astype(float) ** -2.2)
    cdf /= cdf[-1]
    x = d[np.searchsorted(cdf, rng.random(300_000))]
    v, c = np.unique(x, return_counts=True)
    assert ks.fit(v, c)["ks"] < 0.02
    # Kronecker graph with per-level noise: scale-free by the test
    g = gen.rmat(17, 16, seed=2, noise=0.1)
    v, c = odeg.distribution(odeg.degree(g.u, g.v, g.n))
    assert ks.fit(v, c)["ks"] < 0.05
    # lattice and bounded-degree component forest (de Bruijn stand-in): not scale-free
    for g in [gen.grid(400, 0.7, seed=3), gen.plcomp(400_000, seed=3)]:
        v, c = odeg.distribution(odeg.degree(g.u, g.v, g.n))
        assert ks.fit(v, c)["ks"] > 0.1
    # Poisson degrees: the tail is lighter than any power law, alpha hits its bound
    g = gen.gnm(200_000, 800_000, seed=3)
    v, c = odeg.distribution(odeg.degree(g.u, g.v, g.n))
    assert ks.fit(v, c)["alpha"] == ks.ALPHA_HI


def test_no_candidate_gives_inf():
    r = ks.fit(np.array([1, 2]), np.array([3, 4]))
    assert math.isinf(r["ks"]) and not ks.decide_bfs(r["ks"])
    assert ks.decide_bfs(0.0499) and not ks.decide_bfs(0.05)


def test_planted_sign_error_in_derivative_is_caught():
    """A wrong sign in d zeta / ds would break the finite-difference pin."""
    s, q = 2.2, 6.0
    h = 1e-5 * s
    fd = (ss.zeta(s + h, q) - ss.zeta(s - h, q)) / (2 * h)
    assert abs(-float(ks.hurwitz_zeta_ds(s, q)) / fd - 1) > 1.0


def test_observed_only_reading():
    """The two readings of the K-S gap: over every integer of [d_min, d_max]
    (the statistic used) or at the observed degrees only.  The second takes
    the maximum over a subset, so it never exceeds the first; on a support
    without gaps the two coincide; across a gap the integer reading also sees
    the model CDF rise before the next observed degree (worked here by hand:
    alpha = 2, degrees 1 and 10 with 61 and 39 vertices)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        vals = np.unique(rng.integers(1, 400, int(rng.integers(3, 40))))
        cnts = rng.integers(1, 500, vals.shape[0])
        a = ks.fit(vals, cnts)
        b = ks.fit(vals, cnts, observed_only=True)
        if math.isfinite(a["ks"]):
            assert b["ks"] <= a["ks"] + 1e-15
    vals = np.arange(1, 60)
    cnts = np.maximum(1, (1e5 * vals ** -2.2).astype(np.int64))
    assert ks.fit(vals, cnts)["ks"] == ks.fit(vals, cnts, observed_only=True)["ks"]
    vals = np.asarray([1, 10])
    cnts = np.asarray([61, 39])
    z = ss.zeta(2.0, 1.0)
    s1, f1 = 0.61, 1.0 / z                                # S(1), P(D <= 1)
    f9 = 1.0 - ss.zeta(2.0, 10.0) / z                     # P(D <= 9): the model just before 10
    f10 = 1.0 - ss.zeta(2.0, 11.0) / z
    d_int = max(abs(s1 - f1), abs(s1 - f9), abs(1.0 - f10))
    d_obs = max(abs(s1 - f1), abs(1.0 - f10))
    assert abs(ks.ks_distance(vals, cnts, 1, 2.0) - d_int) < 1e-12
    assert abs(ks.ks_distance(vals, cnts, 1, 2.0, observed_only=True) - d_obs) < 1e-12
    assert d_obs < 0.1 < d_int
