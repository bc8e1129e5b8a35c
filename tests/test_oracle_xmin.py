"""Pins of the oracle's law with a lower cutoff xmin (p(k) = k^-alpha /
zeta(alpha, xmin), k >= xmin; the practice the paper cites for fitting power
laws, with xmin = 1 its own case), against what the mathematics fixes:
partial sums of the pmf at high precision, the table search, the law of the
draws including the rejection tail, a grid search of the log-likelihood,
brute-force KS over every integer, the all-at-cutoff rule, and the choice of
xmin on data whose power-law part starts at a known value.
"""
import math

import mpmath as mp
import numpy as np
import pytest


def _Z(a, q):
    with mp.workdps(40):
        return mp.zeta(mp.mpf(a), mp.mpf(q))


def _F_direct(a, xmin, t):
    """F(t) as a partial sum of the pmf (not the Hurwitz difference)."""
    with mp.workdps(40):
        s = mp.fsum(mp.mpf(k) ** (-mp.mpf(a)) for k in range(xmin, t + 1))
        return s / _Z(a, xmin)


def _Zsum(a, q):
    """zeta(a, q) by partial sums for a >= 10 (mpmath's own Hurwitz zeta is
    not accurate at large a); the remainder after 6,000 terms is negligible."""
    with mp.workdps(40):
        return mp.fsum(mp.mpf(k) ** -mp.mpf(a) for k in range(q, q + 6000)) + \
            mp.zeta(a, q + 6000)


@pytest.mark.parametrize("a,xmin", [(1.5, 2), (2.5, 7), (3.3, 100), (1.8, 4000),
                                    (40.0, 17), (25.0, 30), (12.0, 16)])
def test_cdf_table_is_the_partial_sum_of_the_pmf(orc, a, xmin):
    T = orc.hz_cdf_table(a, xmin)
    Z = _Zsum if a >= 10.0 else _Z
    for j in (1, 2, 3, 17, 200, 4096):
        want = float(_F_direct(a, xmin, xmin + j - 1)) if j <= 200 else \
            float(1 - Z(a, xmin + j) / Z(a, xmin))
        assert abs(T[j - 1] - want) < 2e-15, (a, xmin, j)
    assert np.all(np.diff(T) >= 0)


@pytest.mark.parametrize("xmin", [2, 16, 17, 20])
def test_mle_large_root_at_a_small_cutoff(orc, xmin):
    """Samples piled at the cutoff have roots far above 2 (here 6 to 60):
    the fitted exponent solves eq. (2) with partial sums at 40 digits, to
    the FP64 rounding of mu."""
    for extra in ([1, 1, 1], [1, 1, 2], [1] * 6 + [3]):
        x = np.array([xmin] * 60 + [xmin + e for e in extra])
        r = orc.hz_fit(x, xmin)
        a = r["alpha_hat"]
        assert not (r["flags"] & orc.FLAG_NOCONV) and a > 5.0, (xmin, extra, a)
        with mp.workdps(40):
            w = [(mp.mpf(k) ** -mp.mpf(a), mp.log(k)) for k in range(xmin, xmin + 6000)]
            mu = mp.fsum(t * l for t, l in w) / mp.fsum(t for t, _ in w)
        m = r["S"] / x.size
        assert abs(float(mu) - m) <= 8 * 2.0 ** -53 * m, (xmin, extra, float(mu), m)


def test_xmin_one_is_the_pure_law(orc):
    assert np.array_equal(orc.hz_cdf_table(2.2, 1), orc.cdf_table(2.2))
    rng = np.random.default_rng(4)
    for _ in range(5):
        x = rng.zipf(1.9, size=int(rng.integers(2, 60)))
        r, p = orc.hz_fit(x, 1), orc.fit(x)
        assert (r["alpha_hat"], r["D"], r["S"], r["flags"]) == (p["alpha_hat"], p["D"], p["S"], p["flags"])
    assert np.array_equal(orc.hz_sample(2.5, 1, 50, 3, 4, 5)[0], orc.sample(2.5, 50, 3, 4, 5)[0])


def test_draws_are_the_table_search_shifted(orc):
    for a, xmin in [(2.5, 3), (1.7, 50)]:
        T = orc.hz_cdf_table(a, xmin)
        x, _ = orc.hz_sample(a, xmin, 401, 9, 2, 11)
        for i in range(401):
            w = orc.philox([i >> 1, 11, 2, 0], [9, 0])
            U = orc.u53(w[2], w[3]) if i & 1 else orc.u53(w[0], w[1])
            if U <= T[-1]:
                assert x[i] == xmin - 1 + int(np.searchsorted(T, U, side="left")) + 1
            else:
                assert x[i] >= xmin + 4096
        assert x.min() >= xmin


def test_draws_follow_the_law_including_the_tail(orc):
    """alpha = 1.6, xmin = 500: P(X >= xmin + 4096) is about 0.26, so the
    rejection tail is exercised heavily; chi-square on bins whose exact
    probabilities are Hurwitz differences."""
    from scipy import stats
    a, xmin = 1.6, 500
    x = np.concatenate([orc.hz_sample(a, xmin, 2000, 21, 0, r)[0] for r in range(4)])
    edges = [xmin, xmin + 1, xmin + 3, xmin + 10, xmin + 50, xmin + 300, xmin + 1500,
             xmin + 4096, xmin + 10000, xmin + 50000, xmin + 500000, 10 ** 18]
    Zx = _Z(a, xmin)
    p = np.array([float((_Z(a, lo) - _Z(a, hi)) / Zx) for lo, hi in zip(edges[:-1], edges[1:])])
    obs = np.histogram(x, bins=np.array(edges, dtype=np.float64))[0]
    chi2 = ((obs - p * x.size) ** 2 / (p * x.size)).sum()
    assert p[-4:].sum() > 0.25
    assert stats.chi2.sf(chi2, len(p) - 1) > 1e-3, (obs, p * x.size)


def test_mle_grid_search_of_loglikelihood(orc):
    rng = np.random.default_rng(8)
    for xmin in (2, 10, 300):
        for _ in range(3):
            x = xmin - 1 + rng.zipf(2.1, size=int(rng.integers(5, 40)))
            r = orc.hz_fit(x, xmin)
            S, n = r["S"], r["n_tail"]
            with mp.workdps(30):
                ll = lambda g: float(-g * S - n * mp.log(mp.zeta(g, xmin)))  # noqa: E731
                if r["flags"] & orc.FLAG_NOCONV:
                    # the likelihood still rises at the bracket end 64
                    assert r["alpha_hat"] == 64.0 and ll(64.0) > ll(63.9), (xmin, x)
                    continue
                grid = np.linspace(max(1.02, r["alpha_hat"] - 0.6), r["alpha_hat"] + 0.6, 121)
                best = grid[int(np.argmax([ll(g) for g in grid]))]
                lo, hi = best - 0.01, best + 0.01
                for _ in range(50):
                    c = hi - (hi - lo) / 1.618033988749895
                    d = lo + (hi - lo) / 1.618033988749895
                    if ll(c) > ll(d):
                        hi = d
                    else:
                        lo = c
            assert abs(0.5 * (lo + hi) - r["alpha_hat"]) < 1e-6, (xmin, x)


def test_mle_root_above_the_bracket(orc):
    """A sample at xmin = 300 with few values above it has its root above 64."""
    x = np.array([300] * 12 + [301, 303])
    r = orc.hz_fit(x, 300)
    assert r["flags"] & orc.FLAG_NOCONV and r["alpha_hat"] == 64.0
    with mp.workdps(30):
        mu64 = -mp.zeta(64, 300, derivative=1) / mp.zeta(64, 300)
    assert float(mu64) > r["S"] / 14


def test_mle_solves_the_likelihood_equation(orc):
    for xmin, m_over in [(5, 0.3), (40, 0.05), (1000, 0.4), (12000, 0.7)]:
        m = math.log(xmin) + m_over
        a, f = orc.hz_mle(m, xmin)
        assert f & orc.FLAG_NOCONV == 0
        with mp.workdps(40):
            mu = -mp.zeta(a, xmin, derivative=1) / mp.zeta(a, xmin)
        assert abs(float(mu) - m) < 1e-13 * m, (xmin, a)


def test_values_below_cutoff_are_ignored(orc):
    x = np.array([1, 2, 2, 3, 5, 8, 13, 21, 34, 55, 89, 4, 6, 9])
    r = orc.hz_fit(x, 5)
    s = orc.hz_fit(x[x >= 5], 5)
    assert r == s and r["n_tail"] == 9
    with pytest.raises(ValueError):
        orc.hz_fit(x, 90)
    with pytest.raises(ValueError):
        orc.hz_fit(np.array([0, 5]), 5)


def test_all_at_cutoff_rule(orc):
    """Every value equal to xmin: the likelihood has no finite maximum; one
    value is counted as xmin + 1 (the pure law's all-ones rule at xmin = 1)."""
    for xmin, n in [(2, 10), (7, 3), (100, 25)]:
        r = orc.hz_fit(np.full(n, xmin), xmin)
        assert r["flags"] & orc.FLAG_ALL_ONES
        assert abs(r["S"] - ((n - 1) * math.log(xmin) + math.log(xmin + 1))) < 1e-12 * r["S"]
        with mp.workdps(40):
            mu = -mp.zeta(r["alpha_hat"], xmin, derivative=1) / mp.zeta(r["alpha_hat"], xmin)
        if r["flags"] & orc.FLAG_NOCONV:  # root above 64 (xmin = 100: about 2,500)
            assert r["alpha_hat"] == 64.0 and float(mu) > r["S"] / n
        else:
            assert abs(float(mu) - r["S"] / n) < 1e-13 * r["S"] / n
        # D is the mass above xmin under the fit: all the sample sits at xmin
        with mp.workdps(40):
            want = 1 - float(mp.mpf(xmin) ** (-r["alpha_hat"]) / mp.zeta(r["alpha_hat"], xmin))
        assert abs(r["D"] - want) < 1e-14


def test_ks_bruteforce(orc):
    rng = np.random.default_rng(5)
    for xmin in (3, 20):
        for _ in range(4):
            x = xmin - 1 + rng.zipf(1.8, size=int(rng.integers(3, 25)))
            x = np.minimum(x, xmin + 400)
            r = orc.hz_fit(x, xmin)
            a = r["alpha_hat"]
            xs = np.sort(x)
            with mp.workdps(40):
                Z = mp.zeta(a, xmin)
                F = mp.mpf(0)
                best = mp.mpf(0)
                for t in range(xmin, int(xs[-1]) + 2):
                    F += mp.mpf(t) ** (-mp.mpf(a)) / Z
                    Sn = mp.mpf(int(np.searchsorted(xs, t, side="right"))) / len(x)
                    best = max(best, abs(F - Sn))
            assert abs(r["D"] - float(best)) < 1e-14, (xmin, x)


def test_scan_finds_the_start_of_the_power_law(orc):
    """3,000 values uniform on 1..59 below 5,000 draws of the law with
    cutoff 60: the KS-minimising candidate lies near 60, and its fit recovers
    the exponent."""
    rng = np.random.default_rng(17)
    body = rng.integers(1, 60, size=3000)
    tail = np.concatenate([orc.hz_sample(2.5, 60, 1000, 5, 0, r)[0] for r in range(5)])
    x = np.concatenate([body, tail])
    cand = np.arange(1, 121)
    r = orc.hz_scan(x, cand)
    best = int(cand[r["best"]])
    assert 50 <= best <= 75, best
    assert abs(r["alpha_hat"][r["best"]] - 2.5) < 0.1
    assert r["D"][r["best"]] == r["D"].min()
    # every candidate's fit is the plain fit at that cutoff
    for c in (1, 30, 60, 119):
        f = orc.hz_fit(x, c)
        assert (f["alpha_hat"], f["D"]) == (r["alpha_hat"][c - 1], r["D"][c - 1])
    # a candidate above every value gets D = inf and is never chosen
    r2 = orc.hz_scan(np.array([5, 6, 9]), [5, 10])
    assert r2["best"] == 0 and math.isinf(r2["D"][1])


def test_scan_ties_take_the_first(orc):
    x = np.array([4, 4, 4, 4])
    r = orc.hz_scan(x, [2, 3, 4])  # the same tail {4,4,4,4} at cutoffs 2, 3 differ
    assert r["best"] == int(np.argmin(r["D"]))
    r = orc.hz_scan(x, [4, 4])
    assert r["best"] == 0


def test_simulated_exponents_centre_on_alpha(orc):
    """Consistency of the MLE under the law with cutoff: the mean of
    alpha_hat over 400 replicates of n = 2,000 is within 4 standard errors."""
    for a, xmin in [(2.2, 5), (3.0, 50)]:
        r = orc.hz_simulate(a, xmin, 2000, 3, 1, 0, 400)
        m, se = r["alpha_hat"].mean(), r["alpha_hat"].std(ddof=1) / 20
        assert abs(m - a) < 4 * se + 1e-3, (a, xmin, m, se)
        assert np.all(r["xmax"] >= xmin)


@pytest.mark.parametrize("xmin", [10 ** 5, 10 ** 6, 10 ** 9, 2 ** 40])
def test_mle_at_huge_cutoffs(orc, xmin):
    """Cutoffs up to 2^40: q^-s underflows in FP64 from q of about 6.5e4 at
    s = 64, which the bracket check and the iteration reach; the sums are
    kept scaled by xmin^s.  The root matches mpmath's (its error there is the
    FP64 rounding of m, about ulp(ln xmin)/d^2 for m = ln xmin + d)."""
    lx = math.log(xmin)
    for d in (0.1, 0.67, 2.0):
        a, f = orc.hz_mle(lx + d, xmin)
        with mp.workdps(40):
            mm = mp.mpf(lx) + mp.mpf(d)
            root = mp.findroot(lambda s: -mp.zeta(s, xmin, 1) / mp.zeta(s, xmin) - mm, 1 + 1 / d)
        tol = 1e-13 + 4 * 2.0 ** -53 * lx / d ** 2
        assert not (f & orc.FLAG_NOCONV) and abs(a - float(root)) <= tol * float(root), (xmin, d, a)


def _em40(a, q, P=10):
    """zeta(a, q) by Euler-Maclaurin at 40 digits (q large: converges at once)."""
    with mp.workdps(40):
        a, q = mp.mpf(a), mp.mpf(q)
        acc = q ** (1 - a) / (a - 1) + q ** (-a) / 2
        poch = a
        for i in range(1, P + 1):
            acc += mp.bernoulli(2 * i) / mp.factorial(2 * i) * poch * q ** (-a - 2 * i + 1)
            poch *= (a + 2 * i - 1) * (a + 2 * i)
        return acc


@pytest.mark.parametrize("a,xmin", [(30.0, 10 ** 6), (2.5, 2 ** 40), (64.0, 10 ** 9)])
def test_cdf_table_at_huge_cutoffs(orc, a, xmin):
    T = orc.hz_cdf_table(a, xmin)
    with mp.workdps(40):
        Z = _em40(a, xmin)
        for j in (1, 2, 5, 100, 4096):
            want = 1 - _em40(a, xmin + j) / Z
            assert abs(T[j - 1] - float(want)) < 4e-15, (a, xmin, j, T[j - 1], float(want))
    assert np.all(np.diff(T) >= 0)
