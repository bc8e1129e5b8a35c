"""Pins of the CPU oracle against things other than itself.

Each test ties one part of the oracle to a fact fixed by the paper or by
mathematics: closed forms, arbitrary-precision values (mpmath), an independent
Philox implementation (rocRAND's engine, compiled for the host), brute force on
tiny inputs, invariants, and the values printed in Table 1 of Rappos & Robert
(2013).  They are chosen so that a plausible slip anywhere in the oracle (a
dropped Euler-Maclaurin term, a wrong sign in zeta', an off-by-one in the
quantile index, a '>' for '>=' in the sampler) fails at least one of them.
"""
import math
import shutil
import subprocess
from pathlib import Path

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

GOLDEN = Path(__file__).resolve().parent / "golden"
mp.mp.dps = 40


def _zmp(s, q=1, k=0):
    """mpmath Hurwitz zeta with enough working precision: at large s its
    algorithm cancels, so 40 digits are not enough there (checked against a
    direct Euler-Maclaurin sum done in mpmath at 50 digits)."""
    with mp.workdps(400):
        return mp.zeta(mp.mpf(s), mp.mpf(q), k)


# --------------------------------------------------------------------------
# Philox4x32-10 and the 53-bit uniform
# --------------------------------------------------------------------------
ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(hipcc).exists():
        pytest.skip("hipcc not available to build the rocRAND host probe")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = d / "probe"
    subprocess.run([hipcc, "-O1", "-I/opt/rocm/include", "-x", "hip",
                    "--offload-arch=gfx950", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand_engine(orc, rocrand_probe):
    """rocRAND's philox4x32_10 engine seeded with `seed` at subsequence
    c2 | c3<<32 and offset 4*(c0 | c1<<32) starts from counter (c0,c1,c2,c3)
    under key (seed lo, seed hi); its first four outputs are the block."""
    # The engine's offset is a 64-bit count of words, so c1 < 2^30 here.
    rng = np.random.default_rng(1)
    cases = [((0, 0, 0, 0), (0, 0)), ((1, 2, 3, 4), (5, 6)),
             ((0xffffffff, 0x3fffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff))]
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2**32, 4)]
        c[1] >>= 2
        cases.append((tuple(c), tuple(int(v) for v in rng.integers(0, 2**32, 2))))
    lines = []
    for ctr, key in cases:
        seed = key[0] | (key[1] << 32)
        sub = ctr[2] | (ctr[3] << 32)
        off = 4 * (ctr[0] | (ctr[1] << 32))
        lines.append("%d %d %d" % (seed, sub, off))
    out = subprocess.run([str(rocrand_probe)], input="\n".join(lines) + "\n",
                         capture_output=True, text=True, check=True).stdout.split("\n")
    for (ctr, key), line in zip(cases, out):
        want = [int(v) for v in line.split()]
        got = [int(v) for v in orc.philox(ctr, key)]
        assert got == want, (ctr, key)


def test_u53_grid_and_extremes(orc):
    assert orc.u53(0, 0) == 2.0 ** -53
    assert orc.u53(0xffffffff, 0xffffffff) == 1.0 - 2.0 ** -53
    rng = np.random.default_rng(2)
    for hi, lo in rng.integers(0, 2**32, size=(500, 2)):
        w = (int(hi) << 32) | int(lo)
        u = orc.u53(int(hi), int(lo))
        assert u == ((w >> 11) | 1) / 2.0 ** 53
        k = u * 2.0 ** 53
        assert k == int(k) and int(k) % 2 == 1 and 0.0 < u < 1.0


# --------------------------------------------------------------------------
# zeta, zeta', zeta'' and the Hurwitz zeta (Euler-Maclaurin)
# --------------------------------------------------------------------------
def _rel(a, b):
    return abs(a - b) / abs(b)


def test_zeta_closed_forms(orc):
    z2 = orc.zeta3(2.0)
    assert _rel(z2[0], math.pi ** 2 / 6) < 4e-16
    assert _rel(orc.zeta3(4.0)[0], math.pi ** 4 / 90) < 4e-16
    # zeta'(2) = (pi^2/6) (gamma + ln 2 pi - 12 ln A), A = Glaisher's constant
    zp2 = mp.pi ** 2 / 6 * (mp.euler + mp.log(2 * mp.pi) - 12 * mp.log(mp.glaisher))
    assert _rel(z2[1], float(zp2)) < 1e-15


@pytest.mark.parametrize("s", [1.0 + 2.0 ** -20, 1.0001, 1.01, 1.2, 1.5, 1.75, 2.0,
                               2.5, 3.0, 3.5, 4.7, 8.0, 16.6, 32.0, 64.0])
def test_zeta_and_derivatives_vs_mpmath(orc, s):
    got = orc.zeta3(s)
    for k in range(3):
        want = float(_zmp(s, 1, k))
        assert _rel(got[k], want) < 2e-15, (s, k, got[k], want)


@pytest.mark.parametrize("s", [1.05, 1.5, 2.5, 3.9, 10.0, 40.0])
@pytest.mark.parametrize("q", [1.0, 2.0, 16.0, 17.0, 101.0, 4097.0, 1e6, 1e12, 2.0 ** 62])
def test_hurwitz_vs_mpmath(orc, s, q):
    got = orc.hurwitz3(s, q)
    for k in range(3):
        want = float(_zmp(s, q, k))
        if want == 0.0:
            continue
        assert _rel(got[k], want) < 2e-15, (s, q, k, got[k], want)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 2.5, 3.5])
def test_pmf_sums_to_one_and_cdf_increments(orc, alpha):
    """sum_k p(k) = 1 with p(k) = k^-alpha / zeta(alpha) (eq. 1): the partial
    sum to K plus the mpmath tail zeta(alpha, K+1) must give 1, and the CDF's
    increments must be the pmf."""
    z = orc.zeta3(alpha)[0]
    K = 200000
    k = np.arange(1, K + 1, dtype=np.float64)
    head = math.fsum((k ** -alpha).tolist())
    tail = float(mp.zeta(alpha, K + 1))
    assert abs((head + tail) / z - 1.0) < 2e-15
    for t in [1, 2, 3, 10, 16, 17, 100, 4096, 4097, 10 ** 6]:
        inc = orc.cdf(alpha, t) - orc.cdf(alpha, t - 1)
        assert abs(inc - t ** -alpha / z) < 3e-16
    assert orc.cdf(alpha, 0) == 0.0
    surv = float(mp.zeta(alpha, 10 ** 12 + 1) / mp.zeta(alpha))
    assert abs((1.0 - orc.cdf(alpha, 10 ** 12)) - surv) < 2e-16


@pytest.mark.parametrize("alpha", [1.2, 2.5, 3.5])
def test_cdf_table_values(orc, alpha):
    T = orc.cdf_table(alpha)
    assert T.size == orc.TABLE_H
    assert np.all(np.diff(T) >= 0) and T[-1] < 1.0
    for k in [1, 2, 5, 16, 17, 100, 1000, 4096]:
        want = 1 - mp.zeta(alpha, k + 1) / mp.zeta(alpha)
        assert abs(T[k - 1] - float(want)) <= 3e-16


# --------------------------------------------------------------------------
# Sampler: bit-exact recomputation and the law it produces
# --------------------------------------------------------------------------
def _u53_py(hi, lo):
    w = (int(hi) << 32) | int(lo)
    return ((w >> 11) | 1) / 2.0 ** 53


def _tail_py(orc, alpha, seed, stream, rep, i):
    """Tail draw recomputed with mpmath (50 digits) for the floor."""
    beta = alpha - 1.0
    m = 4097.0
    key = (seed & 0xffffffff, seed >> 32)

    def g(kk):
        return 1.0 / (-kk * math.expm1(-beta * math.log1p(1.0 / kk)))

    for attempt in range(1000):
        w = orc.philox((i, rep, stream, 0x80000000 | attempt), key)
        V, W = _u53_py(w[0], w[1]), _u53_py(w[2], w[3])
        with mp.workdps(50):
            Y = mp.mpf(m) * mp.power(mp.mpf(V), -1 / mp.mpf(beta))
            if Y >= mp.mpf(2) ** 63:
                continue
            X = int(mp.floor(Y))
        if W * g(m) <= g(float(X)):
            return X
    raise AssertionError("no acceptance")


@pytest.mark.parametrize("alpha,n,reps", [(2.5, 400, 3), (1.5, 300, 2), (1.2, 200, 2),
                                          (3.5, 64, 2)])
def test_sampler_recomputed_independently(orc, alpha, n, reps):
    """Every draw equals searchsorted(T, U, 'left') + 1 (the '>=' rule) for
    body draws and the mpmath floor of the Pareto proposal for tail draws."""
    seed, stream = 0x1234_5678_9abc, 7
    T = orc.cdf_table(alpha)
    key = (seed & 0xffffffff, seed >> 32)
    ntail = 0
    for rep in range(reps):
        x, _ = orc.sample(alpha, n, seed, stream, rep)
        for i in range(n):
            w = orc.philox((i >> 1, rep, stream, 0), key)
            U = _u53_py(w[0], w[1]) if i % 2 == 0 else _u53_py(w[2], w[3])
            if U <= T[-1]:
                assert x[i] == np.searchsorted(T, U, side="left") + 1
            else:
                ntail += 1
                assert x[i] == _tail_py(orc, alpha, seed, stream, rep, i)
    if alpha <= 1.5:
        assert ntail > 0


@pytest.mark.parametrize("alpha", [1.2, 1.5, 2.5, 3.5])
def test_sampler_chi_square_vs_exact_pmf(orc, alpha):
    """Draws follow p(k) = k^-alpha/zeta(alpha) restricted to k < 2^63,
    including the rejection tail beyond the table (bins up to 2^63)."""
    n = 200000
    x, _ = orc.sample(alpha, n, 99, 3, 0)
    edges = list(range(1, 33)) + [2 ** j for j in range(6, 64)]
    z = mp.zeta(alpha)
    norm = 1 - mp.zeta(alpha, mp.mpf(2) ** 63) / z

    def sf(a):  # P(X >= a) under the capped law
        return (mp.zeta(alpha, a) - mp.zeta(alpha, mp.mpf(2) ** 63)) / z / norm

    probs = [float(sf(a) - sf(b)) for a, b in zip(edges[:-1], edges[1:])]
    probs.append(float(sf(edges[-1])))
    xs = np.asarray(x, dtype=np.float64)
    idx = np.searchsorted(np.asarray(edges, dtype=np.float64), xs, side="right") - 1
    counts = np.bincount(idx, minlength=len(probs)).astype(float)
    exp = np.asarray(probs) * n
    # merge sparse bins from the right
    obs_m, exp_m, acc_o, acc_e = [], [], 0.0, 0.0
    for o, e in zip(counts[::-1], exp[::-1]):
        acc_o += o
        acc_e += e
        if acc_e >= 20:
            obs_m.append(acc_o)
            exp_m.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        obs_m[-1] += acc_o
        exp_m[-1] += acc_e
    chi2 = sum((o - e) ** 2 / e for o, e in zip(obs_m, exp_m))
    pval = stats.chi2.sf(chi2, len(obs_m) - 1)
    assert pval > 1e-4, (alpha, chi2, len(obs_m))


# --------------------------------------------------------------------------
# MLE (eq. 2)
# --------------------------------------------------------------------------
def test_mle_closed_form_at_two(orc):
    m = -(mp.pi ** 2 / 6 * (mp.euler + mp.log(2 * mp.pi) - 12 * mp.log(mp.glaisher))) \
        / (mp.pi ** 2 / 6)
    a, _ = orc.mle(float(m))
    assert abs(a - 2.0) < 4e-15


def _mle_mp(m):
    """Root of -zeta'(a)/zeta(a) = m by plain bisection at 40 digits (the
    function is decreasing in a); 110 halvings of [1 + 1e-7, 64]."""
    m = mp.mpf(m)
    lo, hi = mp.mpf("1.0000001"), mp.mpf(64)
    for _ in range(110):
        mid = (lo + hi) / 2
        if -mp.zeta(mid, 1, 1) / mp.zeta(mid) - m > 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


@pytest.mark.parametrize("m", [40.0, 5.0, 1.3, 0.57, 0.2, 0.0693, 0.01, 6.9e-6])
def test_mle_vs_mpmath_root(orc, m):
    a, _ = orc.mle(m)
    want = float(_mle_mp(mp.mpf(m)))
    assert _rel(a, want) < 1e-14


def test_mle_grid_search_tiny_samples(orc):
    """alpha_hat maximises l(a) = -a S - n ln zeta(a) (brute-force grid)."""
    rng = np.random.default_rng(5)
    for _ in range(6):
        n = int(rng.integers(3, 12))
        x = rng.zipf(2.2, size=n).astype(np.int64)
        if np.all(x == 1):
            x[0] = 2
        r = orc.fit(x)
        S, ahat = r["S"], r["alpha_hat"]
        ll = lambda a: -a * S - n * mp.log(mp.zeta(a))  # noqa: E731
        grid = np.linspace(1.02, 12.0, 2000)
        vals = [float(ll(g)) for g in grid]
        g0 = grid[int(np.argmax(vals))]
        assert abs(g0 - ahat) < (grid[1] - grid[0])
        for d in (1e-6, 1e-4):
            assert ll(ahat) >= ll(ahat + d) and ll(ahat) >= ll(ahat - d)


def test_all_ones_atoms_match_table1(orc):
    """All-ones samples: S := ln 2, alpha_hat solves -zeta'/zeta = ln2/n and
    D = 1 - 1/zeta(alpha_hat).  These atoms are the values Table 1 prints at
    (N=10: gamma 3.5 q.90, gamma 4 q.90/q.95) and (N=20: gamma 4 q.90)."""
    golden = _table1()
    for n, cells in [(10, [(3.5, 0), (4.0, 0), (4.0, 1)]), (20, [(4.0, 0)])]:
        r = orc.fit(np.ones(n, dtype=np.int64))
        assert r["flags"] & orc.FLAG_ALL_ONES
        assert r["S"] == math.log(2.0)
        want_a = float(_mle_mp(mp.log(2) / n))
        assert _rel(r["alpha_hat"], want_a) < 1e-14
        assert abs(r["D"] - (1 - 1 / float(mp.zeta(want_a)))) < 1e-15
        for g, qi in cells:
            assert round(r["D"], 4) == golden[(g, n)][qi]
    assert abs(orc.fit(np.ones(10, dtype=np.int64))["alpha_hat"] - 3.9040855806) < 1e-9
    assert abs(orc.fit(np.ones(20, dtype=np.int64))["alpha_hat"] - 4.7173769904) < 1e-9


# --------------------------------------------------------------------------
# KS distance (eq. 3)
# --------------------------------------------------------------------------
def _ks_brute(x, a):
    x = np.sort(x)
    n = len(x)
    z = mp.zeta(a)
    best = mp.mpf(0)
    F = mp.mpf(0)
    for t in range(1, int(x[-1]) + 60):
        F += mp.mpf(t) ** (-a) / z
        Sn = mp.mpf(int(np.searchsorted(x, t, side="right"))) / n
        best = max(best, abs(F - Sn))
    return float(best)


def test_ks_bruteforce_tiny_samples(orc):
    rng = np.random.default_rng(11)
    samples = [np.array([1, 1, 1, 2, 5, 5, 9]), np.array([3, 3, 3]),
               np.array([1, 2, 3, 4, 5, 6, 7, 8]), np.array([2, 40, 41, 300]),
               np.array([1] * 20 + [2])]
    for _ in range(8):
        samples.append(np.minimum(rng.zipf(1.8, size=int(rng.integers(2, 30))), 800))
    for x in samples:
        x = x.astype(np.int64)
        r = orc.fit(x)
        assert abs(r["D"] - _ks_brute(x, r["alpha_hat"])) < 1e-14, x


# --------------------------------------------------------------------------
# Quantile rule and Table 1 (statistical)
# --------------------------------------------------------------------------
def test_quantile_index_rule(orc):
    rng = np.random.default_rng(3)
    for R in [1, 2, 7, 10, 99, 100, 1001, 50000]:
        D = np.round(rng.random(R), 2)  # many ties
        s = np.sort(D)
        for num, den in [(9, 10), (95, 100), (99, 100), (999, 1000), (0, 1), (1, 2)]:
            assert orc.quantile(D, num, den) == s[(R * num) // den]
    assert [(50000 * a) // b for a, b in [(9, 10), (95, 100), (99, 100), (999, 1000)]] \
        == [45000, 47500, 49500, 49950]


def _table1():
    out = {}
    for line in (GOLDEN / "table1_pure_zipf.txt").read_text().splitlines():
        if line.startswith("#") or not line.strip():
            continue
        g, n, *q = line.split()
        out[(float(g), int(n))] = [float(v) for v in q]
    return out


@pytest.mark.parametrize("alpha,n,R,tol", [(3.5, 10, 50000, 0.00005), (2.5, 100, 20000, 0.0012),
                                           (2.0, 1000, 4000, 0.0010), (3.0, 50, 20000, 0.0015)])
def test_table1_statistical(orc, alpha, n, R, tol):
    """Quantiles 0.90 / 0.95 within Monte-Carlo error of Table 1 (gamma >= 1.75:
    the paper's gamma <= 1.5 cells are not reproducible by an exact sampler)."""
    want = _table1()[(alpha, n)]
    r = orc.simulate(alpha, n, 2024, 0, 0, R)
    for qi, (num, den) in enumerate([(9, 10), (95, 100)]):
        got = orc.quantile(r["D"], num, den)
        assert abs(got - want[qi]) <= tol, (alpha, n, qi, got, want[qi])


# --------------------------------------------------------------------------
# Parametric bootstrap p-value
# --------------------------------------------------------------------------
def test_bootstrap_equals_fraction_of_simulated_D(orc):
    rng = np.random.default_rng(8)
    x = rng.zipf(2.3, size=150).astype(np.int64)
    r = orc.bootstrap_pvalue(x, 500, 77, 5)
    sim = orc.simulate(r["alpha_hat"], x.size, 77, 5, 0, 500)
    assert r["p_value"] == np.mean(sim["D"] >= r["D"])
    f = orc.fit(x)
    assert r["alpha_hat"] == f["alpha_hat"] and r["D"] == f["D"]


def test_bootstrap_all_ones_counts_ties(orc):
    """All-ones data: every all-ones bootstrap replicate has exactly D_obs,
    and ties count (>=), so p is at least the all-ones fraction."""
    x = np.ones(10, dtype=np.int64)
    r = orc.bootstrap_pvalue(x, 2000, 3, 1)
    sim = orc.simulate(r["alpha_hat"], 10, 3, 1, 0, 2000)
    all_ones = np.mean(sim["flags"] & orc.FLAG_ALL_ONES > 0)
    assert all_ones > 0.3
    assert r["p_value"] >= all_ones


def test_bootstrap_pvalues_uniform_under_null(orc):
    rng = np.random.default_rng(21)
    ps = []
    for k in range(120):
        x = rng.zipf(2.5, size=300).astype(np.int64)
        ps.append(orc.bootstrap_pvalue(x, 200, 1000 + k, k)["p_value"])
    assert stats.kstest(ps, "uniform").pvalue > 1e-3


def test_fit_rejects_invalid(orc):
    with pytest.raises(ValueError):
        orc.fit(np.array([1, 0, 3], dtype=np.int64))
    with pytest.raises(ValueError):
        orc.fit(np.array([], dtype=np.int64))
