"""CPU checks of the library's scalar arithmetic (zpl_math.hpp compiled for
the host) against the oracle and mpmath: Philox, the exact tail floor with
its double-double path, the CDF table, zeta and the MLE.  These validate the
logic the kernels inline; GPU parity is checked separately."""
import ctypes as C
import math
import shutil
import subprocess
from pathlib import Path

import mpmath as mp
import numpy as np
import pytest

HERE = Path(__file__).resolve().parent


@pytest.fixture(scope="module")
def hm(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(hipcc).exists():
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("hm") / "libhm.so"
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    str(HERE / "hostprobe" / "hostmath.cpp"), "-o", str(out)],
                   check=True, capture_output=True)
    L = C.CDLL(str(out))
    P = C.POINTER
    L.hm_philox.argtypes = [P(C.c_uint32)] * 3
    L.hm_tail.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                          P(C.c_uint32)]
    L.hm_tail.restype = C.c_int64
    L.hm_mle.argtypes = [C.c_double, P(C.c_uint32)]
    L.hm_mle.restype = C.c_double
    L.hm_zeta3.argtypes = [C.c_double, P(C.c_double)]
    L.hm_table.argtypes = [C.c_double, P(C.c_double)]
    L.hm_survival.argtypes = [C.c_double, C.c_int64]
    L.hm_survival.restype = C.c_double
    L.hm_S.argtypes = [P(C.c_int64), C.c_int64]
    L.hm_S.restype = C.c_double
    L.hm_dd_exp_log.argtypes = [C.c_double, P(C.c_double)]
    L.hm_dd_exp.argtypes = [C.c_double, C.c_double, P(C.c_double)]
    L.hm_guide_pack_all.argtypes = [P(C.c_uint16), C.c_int, C.c_uint64, P(C.c_uint32)]
    L.hm_hurwitz3.argtypes = [C.c_double, C.c_int64, P(C.c_double)]
    L.hm_mle_hz.argtypes = [C.c_double, C.c_int64, P(C.c_uint32)]
    L.hm_mle_hz.restype = C.c_double
    L.hm_tail_from.argtypes = [C.c_double, C.c_int64, C.c_uint64, C.c_uint32, C.c_uint32,
                               C.c_uint32, P(C.c_uint32)]
    L.hm_tail_from.restype = C.c_int64
    L.hm_survival_cut.argtypes = [C.c_double, C.c_int64]
    L.hm_survival_cut.restype = C.c_double
    L.hm_survival_rel.argtypes = [C.c_double, C.c_int64, C.c_int64]
    L.hm_survival_rel.restype = C.c_double
    L.hm_zeta3_trunc.argtypes = [C.c_double, C.c_uint32, P(C.c_double)]
    L.hm_zeta3_trunc_em.argtypes = [C.c_double, C.c_uint32, P(C.c_double)]
    L.hm_moments012.argtypes = [C.c_double, P(C.c_double)]
    L.hm_guide_index.argtypes = [C.c_uint64, C.c_int]
    L.hm_guide_index.restype = C.c_int
    L.hm_guide_refinement.argtypes = [C.c_uint64]
    L.hm_guide_refinement.restype = C.c_int
    L.hm_guide_build.argtypes = [P(C.c_double), P(C.c_uint16)]
    L.hm_guide_build.restype = C.c_int
    L.hm_guide_index_many.argtypes = [P(C.c_uint64), C.c_int64, C.c_int, P(C.c_int32)]
    L.hm_mle_trunc.argtypes = [C.c_double, C.c_uint32, P(C.c_uint32)]
    L.hm_mle_trunc.restype = C.c_double
    for f, args in [("hm_mle_it", [C.c_double]), ("hm_mle_trunc_it", [C.c_double, C.c_uint32]),
                    ("hm_mle_hz_it", [C.c_double, C.c_int64])]:
        getattr(L, f).argtypes = args + [P(C.c_uint32), P(C.c_int)]
        getattr(L, f).restype = C.c_double
    return L


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def test_philox_same_as_oracle(hm, orc):
    rng = np.random.default_rng(4)
    for _ in range(300):
        c = rng.integers(0, 2**32, 4).astype(np.uint32)
        k = rng.integers(0, 2**32, 2).astype(np.uint32)
        out = np.zeros(4, np.uint32)
        hm.hm_philox(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
        assert np.array_equal(out, orc.philox(c, k))


@pytest.mark.parametrize("alpha", [1.2, 1.3, 1.5, 2.5, 3.5])
def test_tail_draws_bit_exact_vs_oracle(hm, orc, alpha):
    """The library's tail sampler (FP64 with a double-double floor near
    integers and above 2^52) returns the oracle's quad-precision floor, for
    every draw index (the tail stream does not depend on the body uniform)."""
    seed, stream = 0xfeedbeef12345, 3
    big = 0
    for rep in range(3):
        for i in range(1500):
            f1 = C.c_uint32(0)
            x_h = hm.hm_tail(alpha, seed, stream, rep, i, C.byref(f1))
            x_o, f_o = orc.tail_draw(alpha, seed, stream, rep, i)
            assert x_h == x_o, (alpha, rep, i, x_h, x_o)
            assert f1.value == f_o
            big += x_h > 2 ** 52
    if alpha == 1.2:
        assert big > 5  # the double-double path above 2^52 was exercised


def test_dd_exp_log_precision(hm):
    out = np.zeros(4)
    for v in [2.0 ** -53, 1e-300, 0.3, 0.999999, 1.5, 7.0, 40.0, 700.0]:
        hm.hm_dd_exp_log(v, _p(out, C.c_double))
        with mp.workdps(60):
            L = mp.log(mp.mpf(v))
            got = mp.mpf(out[0]) + mp.mpf(out[1])
            # near v = 1 the double-double log is accurate in absolute terms
            assert abs(got - L) <= abs(L) * mp.mpf(2) ** -100 + mp.mpf(2) ** -104
            if v < 700:
                E = mp.exp(mp.mpf(v))
                got = mp.mpf(out[2]) + mp.mpf(out[3])
                assert abs(got - E) <= E * mp.mpf(2) ** -100


def test_dd_exp_every_table_entry(hm):
    """dd_exp at double-double arguments (64 q + j) ln2/64 + r for every
    table entry j, exponents q across the tail sampler's range and both
    signs, and |r| up to the reduction bound ln2/128: relative error within
    2^-102 of the 60-digit value."""
    rng = np.random.default_rng(7)
    out = np.zeros(2)
    with mp.workdps(60):
        c = mp.log(2) / 64
        for j in range(64):
            for q in (-1, 0, 1, -11, 9, 50, -57):
                r = (rng.random() - 0.5) * float(c)
                a = (64 * q + j) * c + mp.mpf(r)
                hi = float(a)
                lo = float(a - mp.mpf(hi))
                hm.hm_dd_exp(hi, lo, _p(out, C.c_double))
                E = mp.exp(mp.mpf(hi) + mp.mpf(lo))
                got = mp.mpf(out[0]) + mp.mpf(out[1])
                assert abs(got - E) <= E * mp.mpf(2) ** -102, (j, q, r)


def test_dd_log_over_the_tail_uniforms(hm):
    """dd_log at random odd multiples of 2^-53 (the sampler's V), including
    the smallest: absolute error within 2^-100 |ln V| + 2^-104."""
    rng = np.random.default_rng(11)
    out = np.zeros(4)
    ms = [1, 3, (1 << 53) - 1] + [int(x) | 1 for x in rng.integers(1, 1 << 53, 300)]
    ms += [int(x) | 1 for x in rng.integers(1, 1 << 20, 100)]
    for m in ms:
        v = m * 2.0 ** -53
        hm.hm_dd_exp_log(v, _p(out, C.c_double))
        with mp.workdps(60):
            L = mp.log(mp.mpf(v))
            got = mp.mpf(out[0]) + mp.mpf(out[1])
            assert abs(got - L) <= abs(L) * mp.mpf(2) ** -100 + mp.mpf(2) ** -104, m


@pytest.mark.parametrize("alpha,ulps", [(1.05, 12), (1.2, 4), (1.5, 2), (2.5, 2), (3.5, 1),
                                        (8.0, 1)])
def test_table_within_ulps_of_oracle(hm, orc, alpha, ulps):
    """Both sides round T[k] = 1 - zeta(a,k+1)/zeta(a) independently; the gap
    (in units of 2^-53) grows as alpha -> 1 where zeta(a) ~ 1/(a-1)."""
    T = np.zeros(4096)
    hm.hm_table(alpha, _p(T, C.c_double))
    To = orc.cdf_table(alpha)
    assert np.max(np.abs(T - To)) <= ulps * 2.0 ** -53
    assert np.all(np.diff(T) >= 0)


@pytest.mark.parametrize("s", [1.0 + 2 ** -20, 1.01, 1.5, 2.0, 2.5, 3.9, 8.0, 16.6, 40.0, 64.0])
def test_zeta3_vs_oracle(hm, orc, s):
    out = np.zeros(3)
    hm.hm_zeta3(s, _p(out, C.c_double))
    ref = orc.zeta3(s)
    tol = 1e-15 * max(1.0, s)
    assert np.all(np.abs(out - ref) <= tol * np.abs(ref)), (out, ref)


def test_survival_vs_oracle(hm, orc):
    for a in [1.2, 2.5, 3.5]:
        for v in [0, 1, 5, 15, 16, 17, 100, 4095, 4096, 4097, 10 ** 6, 10 ** 15, 2 ** 63 - 1]:
            got = hm.hm_survival(a, v)
            with mp.workdps(60):
                want = float(mp.zeta(a, mp.mpf(v) + 1))
            # relative error ~ a * ulp(ln v): up to ~1e-14 near v = 2^63
            assert abs(got - want) <= 2e-14 * abs(want) + 1e-300, (a, v, got, want)


@pytest.mark.parametrize("m", [43.0, 5.0, 1.3, 0.57, 0.2, 0.0693, 0.01, 6.9e-6, 1e-9])
def test_mle_vs_oracle(hm, orc, m):
    f = C.c_uint32(0)
    a = hm.hm_mle(m, C.byref(f))
    ao, _ = orc.mle(m)
    assert abs(a - ao) <= 2e-14 * ao
    assert not (f.value & 8)


def test_exact_S_order_independent(hm):
    rng = np.random.default_rng(0)
    x = rng.zipf(1.4, size=5000).astype(np.int64)
    x = np.minimum(x, 2 ** 62)
    s1 = hm.hm_S(_p(x, C.c_int64), x.size)
    y = x[rng.permutation(x.size)].copy()
    s2 = hm.hm_S(_p(y, C.c_int64), y.size)
    assert s1 == s2
    want = math.fsum(np.log(x.astype(np.float64)))
    assert abs(s1 - want) <= 4e-16 * want


@pytest.mark.parametrize("s,q", [(1.3, 2), (2.5, 7), (3.0, 17), (2.2, 18), (4.0, 300),
                                 (50.0, 300), (1.7, 123456),
                                 # large s at small q: the tail starts at 1.6 s + 10
                                 (10.0, 17), (20.0, 17), (40.0, 17), (64.0, 17), (54.0, 16),
                                 (30.0, 2), (25.0, 30), (50.0, 60), (64.0, 106), (64.0, 107)])
def test_hurwitz3_at_a_cutoff(hm, s, q):
    """zeta(s, q) and its s-derivatives for the law with a lower cutoff, each
    multiplied by q^s (the library's scale, a common factor that cancels in
    eq. 2), against partial sums at 40 digits (mpmath's own Hurwitz zeta is
    not accurate enough at s = 50, q = 300) or mpmath where the sum is long."""
    out = np.zeros(3)
    hm.hm_hurwitz3(s, q, _p(out, C.c_double))
    with mp.workdps(40):
        if s >= 10.0:  # the sum converges within a few thousand terms
            K = q + 5000
            terms = [(mp.mpf(k) ** -s, mp.log(k)) for k in range(q, K)]
            want = [mp.fsum(t for t, _ in terms), -mp.fsum(t * l for t, l in terms),
                    mp.fsum(t * l * l for t, l in terms)]
        else:
            want = [mp.zeta(s, q), mp.zeta(s, q, 1), mp.zeta(s, q, 2)]
        want = [w * mp.mpf(q) ** s for w in want]
    # q^-s = exp(-s ln q) inherits s times the rounding of ln q (about
    # s ln(q) 1.1e-16 relative); that factor is common to all three and
    # cancels in zeta'/zeta
    tol = 3e-15 + 1.2e-16 * s * math.log(q)
    for i in range(3):
        assert abs(out[i] - float(want[i])) <= tol * abs(float(want[i])), (s, q, i)


@pytest.mark.parametrize("xmin", [2, 9, 17, 60, 300, 5000])
def test_mle_at_a_cutoff_matches_oracle(hm, orc, xmin):
    rng = np.random.default_rng(xmin)
    for _ in range(6):
        x, _ = orc.hz_sample(float(rng.uniform(1.5, 4.0)), xmin, int(rng.integers(5, 400)), 3,
                             1, int(rng.integers(0, 1000)))
        r = orc.hz_fit(x, xmin)
        if r["flags"] & orc.FLAG_NOCONV:
            continue
        f = C.c_uint32(0)
        a = hm.hm_mle_hz(r["S"] / r["n_tail"], xmin, C.byref(f))
        assert abs(a - r["alpha_hat"]) <= 1e-12 * r["alpha_hat"], (xmin, x)


def test_tail_from_a_cutoff_matches_oracle(hm, orc):
    for a, xmin in [(1.6, 500), (2.5, 3), (1.2, 10 ** 6)]:
        T = orc.hz_cdf_table(a, xmin)
        for i in range(400):
            w = orc.philox([i >> 1, 0, 7, 0], [11, 0])
            U = orc.u53(w[2], w[3]) if i & 1 else orc.u53(w[0], w[1])
            if U <= T[-1]:
                continue
            f = C.c_uint32(0)
            got = hm.hm_tail_from(a, xmin, 11, 7, 0, i, C.byref(f))
            x, _ = orc.hz_sample(a, xmin, i + 1, 11, 7, 0)
            assert got == x[i], (a, xmin, i)


@pytest.mark.parametrize("K", [2, 20, 1000, 4096])
def test_truncated_sums_vs_oracle(hm, orc, K):
    """Z_K and its s-derivatives (the library sums from K down with exp of
    s ln k from a rounded ln k; the oracle with pow): within the
    recursive-summation bound K eps plus the exponent's rounding, |s| ln K
    eps relative per term (the terms of each sum share one sign)."""
    for s in (-3.0, 0.0, 0.25, 1.0, 2.5, 40.0):
        out = (C.c_double * 3)()
        hm.hm_zeta3_trunc(s, K, out)
        ref = orc.tz_norm3(s, K)
        tol = 4e-16 * K + 2.3e-16 * abs(s) * math.log(K)
        for i in range(3):
            assert abs(out[i] - ref[i]) <= tol * abs(ref[i]) + 1e-300, (K, s, i)


def test_moments_of_the_integral(hm):
    """M_k(z) = int_0^1 v^k e^(zv) dv, k = 0..2 (series for |z| <= 2, closed
    forms beyond) against mpmath quadrature at 30 digits, on both sides of
    the switch and at z = 0."""
    mp.mp.dps = 30
    for z in (-300.0, -40.0, -4.0, -2.0000001, -2.0, -1.0, -1e-9, 0.0, 1e-12, 0.5, 1.999999,
              2.0, 2.0000001, 3.0, 50.0, 400.0):
        out = (C.c_double * 3)()
        hm.hm_moments012(z, out)
        for k in range(3):
            ref = mp.quad(lambda v: v ** k * mp.e ** (z * v), [0, 1])
            assert abs(out[k] - float(ref)) <= 4e-16 * abs(float(ref)), (z, k, out[k], ref)


@pytest.mark.parametrize("K", [65, 66, 100, 500, 1000, 4096])
def test_truncated_em_sums_vs_direct(hm, orc, K):
    """Z_K, Z_K', Z_K'' by Euler-Maclaurin above q0 = max(17, ceil(1.6|s| + 10))
    against the oracle's direct sums (pow per term), over the whole exponent
    range, through s = 1 (where the integral term's 1/(1 - s) form is
    singular) and both sides of every q0 step."""
    for s in (-64.0, -40.0, -10.0, -4.375, -3.0, -1.0, -0.5, 0.0, 0.25, 0.999999, 1.0,
              1.000001, 1.5, 2.5, 4.375, 4.376, 10.0, 40.0, 64.0):
        q0 = max(17, math.ceil(1.6 * abs(s) + 10))
        if K < q0 + 48:
            continue
        out = (C.c_double * 3)()
        hm.hm_zeta3_trunc_em(s, K, out)
        ref = orc.tz_norm3(s, K)
        for i in range(3):
            tol = (4e-16 * K + 2.3e-16 * abs(s) * math.log(K) + 2e-15) * abs(ref[i])
            assert abs(out[i] - ref[i]) <= tol + 1e-300, (K, s, i, out[i], ref[i])


def test_truncated_em_sums_vs_mpmath(hm):
    """Z_K(s) and its derivatives at 30 digits (mpmath partial sums), where
    the oracle is not involved."""
    mp.mp.dps = 30
    for K, s in ((1000, 0.5), (1000, 1.0), (1000, 2.5), (4096, -2.0), (300, 7.0)):
        out = (C.c_double * 3)()
        hm.hm_zeta3_trunc_em(s, K, out)
        ks = [mp.mpf(k) for k in range(1, K + 1)]
        ref = [mp.fsum(k ** -s for k in ks), -mp.fsum(mp.log(k) * k ** -s for k in ks),
               mp.fsum(mp.log(k) ** 2 * k ** -s for k in ks)]
        for i in range(3):
            assert abs(out[i] - float(ref[i])) <= 2e-15 * abs(float(ref[i])), (K, s, i)


@pytest.mark.parametrize("K", [2, 20, 1000, 4096])
def test_truncated_mle_vs_oracle(hm, orc, K):
    """mle_alpha_trunc on the mean log of simulated samples (and of samples
    with no root in [-64, 64]) against the oracle's truncated MLE."""
    rng = np.random.default_rng(K)
    for _ in range(8):
        g = float(rng.uniform(-0.5, 4.0))
        x = orc.tz_sample(g, K, int(rng.integers(3, 300)), 5, 2, int(rng.integers(0, 1000)))
        r = orc.tz_fit(x, K)
        f = C.c_uint32(0)
        a = hm.hm_mle_trunc(r["S"] / x.size, K, C.byref(f))
        assert abs(a - r["alpha_hat"]) <= 1e-11 * max(abs(r["alpha_hat"]), 1.0), (K, g, x)
        assert (f.value & 8) == (r["flags"] & 8)
    for m in (0.0 + 1e-300, math.log(K)):  # every value 1 (without the rule) / every value K
        f = C.c_uint32(0)
        a = hm.hm_mle_trunc(m, K, C.byref(f))
        ao, fo = orc.tz_mle(m, K)
        assert a == ao and (f.value & 8) and (fo & 8), (K, m, a, ao)


@pytest.mark.parametrize("a", [3.0, 10.0, 25.0, 40.0, 64.0])
def test_survival_at_a_cutoff_large_exponent(hm, a):
    """zeta(a, v+1) as the law with a cutoff uses it (CDF table and KS),
    against partial sums at 40 digits, for v below, at and above 1.6 a + 10."""
    for v in (1, 2, 5, 15, 16, 17, 18, 30, 60, 100, 111, 112, 200, 5000):
        got = hm.hm_survival_cut(a, v)
        with mp.workdps(40):
            # 6,000 terms, then the remainder (relatively tiny: mpmath's own
            # Hurwitz value is accurate enough for it)
            want = mp.fsum(mp.mpf(k) ** -a for k in range(v + 1, v + 1 + 6000)) + \
                mp.zeta(a, v + 1 + 6000)
            if a < 10.0:
                want = mp.zeta(a, v + 1)
        tol = 3e-15 + 1.2e-16 * a * math.log(v + 1)
        assert abs(got - float(want)) <= tol * float(want), (a, v, got, float(want))


def _var_trunc(a, K):
    with mp.workdps(40):
        w = [mp.mpf(k) ** -mp.mpf(a) for k in range(1, K + 1)]
        Z = mp.fsum(w)
        mu = mp.fsum(mp.log(k) * w[k - 1] for k in range(1, K + 1)) / Z
        return float(mp.fsum((mp.log(k) - mu) ** 2 * w[k - 1] for k in range(1, K + 1)) / Z)


def _var_cut(a, q):
    with mp.workdps(40):
        N = q + 6000  # partial sums: mpmath's own Hurwitz zeta is not accurate at large a
        w = [(mp.mpf(k) ** -mp.mpf(a), mp.log(k)) for k in range(q, N)]
        Z = mp.fsum(t for t, _ in w)
        mu = mp.fsum(t * l for t, l in w) / Z
        return float(mp.fsum(t * (l - mu) ** 2 for t, l in w) / Z)


def test_mle_edges_agree_within_the_conditioning_of_eq2(hm, orc):
    """Across each law's whole range of mean logs m, up to its edges (every
    value at K, or at the cutoff), the library's root agrees with the
    oracle's to 1e-10, or -- where eq. (2) is ill-conditioned -- within
    4 eps m / Var(ln X) at the root: an FP64 mu is only that precise, and
    both sides sit at that noise.  (This found the Euler-Maclaurin start
    that the law with a cutoff needs at large exponents.)"""
    eps = 2.0 ** -53
    rng = np.random.default_rng(23)
    for K in (2, 3, 20, 1000):
        lnK = math.log(K)
        ms = list(rng.uniform(0, lnK, 25)) + [lnK * (1 - 10.0 ** -e) for e in (2, 5, 8, 11, 14)]
        for m in ms:
            f = C.c_uint32(0)
            a = hm.hm_mle_trunc(m, K, C.byref(f))
            ao, fo = orc.tz_mle(m, K)
            if abs(a - ao) <= 1e-10 * max(abs(ao), 1.0):
                continue
            assert abs(ao) < 64.0, (K, m, a, ao)
            assert abs(a - ao) <= 4 * eps * m / _var_trunc(ao, K), (K, m, a, ao)
    for xmin in (2, 3, 16, 17, 18, 30, 100):
        lx = math.log(xmin)
        for d in list(10 ** rng.uniform(-12, 1.2, 25)):
            m = lx + d
            f = C.c_uint32(0)
            a = hm.hm_mle_hz(m, xmin, C.byref(f))
            ao, fo = orc.hz_mle(m, xmin)
            if abs(a - ao) <= 1e-10 * ao:
                continue
            assert ao < 64.0, (xmin, m, a, ao)
            assert abs(a - ao) <= 4 * eps * m / _var_cut(ao, xmin), (xmin, m, a, ao)


def _zeta_rel(a, v, x):
    """zeta(a, v+1) x^a in 40 digits: partial sum to v + 6001, then the
    Euler-Maclaurin remainder (exact to far below FP64 there)."""
    with mp.workdps(40):
        a, q = mp.mpf(a), mp.mpf(v + 1)
        M = q + 6000
        head = mp.fsum((mp.mpf(k) / x) ** -a for k in range(v + 1, v + 6001))
        tail = (M / x) ** -a * (M / (a - 1) + mp.mpf(1) / 2 + a / (12 * M))
        return head + tail


@pytest.mark.parametrize("a,xmin", [(2.5, 10**5), (30.0, 10**6), (64.0, 10**9),
                                    (1.5, 2**40), (12.0, 4097)])
def test_survival_relative_to_a_huge_cutoff(hm, a, xmin):
    """zeta(a, v+1) xmin^a, the scaled survival the law with a cutoff above 17
    uses, against 40 digits at v = xmin - 1 (the normaliser) and above: it
    stays O(xmin/(a-1)) where xmin^-a itself underflows FP64."""
    for v in (xmin - 1, xmin, xmin + 5, xmin + 150, 2 * xmin):
        got = hm.hm_survival_rel(a, v, xmin)
        ref = _zeta_rel(a, v, xmin)
        assert abs(got - float(ref)) <= 4e-15 * float(ref), (a, xmin, v, got, ref)


@pytest.mark.parametrize("xmin", [10**5, 10**6, 10**9, 2**40])
def test_mle_at_huge_cutoffs_agrees_with_the_oracle(hm, orc, xmin):
    """Eq. (2) for the law with a cutoff far above where x^-64 underflows
    FP64 (xmin = 1e5 .. 2^40): the library's root agrees with the oracle's
    within the conditioning bound 4 eps m / Var(ln X) (Var of ln X is about
    1/(a-1)^2, so the root is ill-conditioned in proportion to ln xmin),
    converges without flags, and the bracket end 64 is not returned."""
    eps = 2.0 ** -53
    lx = math.log(xmin)
    for d in (0.05, 0.3, 0.67, 2.0, 8.0):
        m = lx + d
        f = C.c_uint32(0)
        a = hm.hm_mle_hz(m, xmin, C.byref(f))
        ao, fo = orc.hz_mle(m, xmin)
        assert f.value & 8 == 0 and fo & 8 == 0, (xmin, d, f.value, fo)
        assert a < 60.0, (xmin, d, a)
        var = 1.0 / (ao - 1.0) ** 2
        assert abs(a - ao) <= max(1e-10 * ao, 4 * eps * m / var), (xmin, d, a, ao)


def test_noconv_agrees_near_the_edges(hm, orc):
    """Close to the edge of each law's range of m (every value at xmin, or at
    K) eq. 2 fixes the root only to about eps m / Var(ln X), coarser than the
    2^-40 step test, and a solver may run to its iteration limit.  Both then
    flag NOCONV (bit 8) only if the last residual of eq. 2 exceeds the
    rounding noise of an FP64 mu (2^-44 m), so the flag means the same on
    both sides: no root found, never rounding noise (before, about one case
    in ten near these edges was flagged on one side only)."""
    rng = np.random.default_rng(8)
    for xmin in (2, 3, 16, 30, 10**6):
        lx = math.log(xmin)
        for d in 10 ** rng.uniform(-14, 1.2, 150):
            f = C.c_uint32(0)
            a = hm.hm_mle_hz(lx + d, xmin, C.byref(f))
            ao, fo = orc.hz_mle(lx + d, xmin)
            assert f.value & 8 == fo & 8, (xmin, d, a, ao, f.value, fo)
    for K in (2, 3, 5, 4097):
        lnK = math.log(K)
        for e in rng.uniform(1, 16, 150):
            m = lnK * (1 - 10.0 ** -e)
            f = C.c_uint32(0)
            a = hm.hm_mle_trunc(m, K, C.byref(f))
            ao, fo = orc.tz_mle(m, K)
            assert f.value & 8 == fo & 8, (K, e, a, ao, f.value, fo)


def test_both_solvers_reach_the_cap_and_agree(hm, orc):
    """The three laws share one stopping rule on both sides: at most 200
    Newton iterations, and NOCONV at that cap only when the last residual of
    eq. 2 exceeds 2^-44 m.  Pinned where both the library's solver and the
    oracle's run into the cap: close to the edge m -> ln K (truncated law,
    K = 2..6) or m -> ln xmin (the law with a cutoff, xmin = 2..4), where an
    FP64 mu fixes the root more coarsely than the step test.  There both
    count exactly 200 iterations, neither flags NOCONV (the residual is
    rounding noise), and the roots agree within the conditioning bound.  The
    pure law's solver never reaches the cap over its whole range of m."""
    eps = 2.0 ** -53
    rng = np.random.default_rng(1)
    both = 0
    for K in (2, 3, 4, 5, 6):
        lnK = math.log(K)
        for e in rng.uniform(1, 17, 600):
            m = lnK * (1 - 10.0 ** -e)
            f, it = C.c_uint32(0), C.c_int(0)
            a = hm.hm_mle_trunc_it(m, K, C.byref(f), C.byref(it))
            ao, fo = orc.tz_mle(m, K)
            io = orc.mle_last_iters()
            assert it.value <= 200 and io <= 200
            assert f.value & 8 == fo & 8, (K, m, a, ao)
            if it.value == 200 and io == 200:
                both += 1
                assert fo & 8 == 0, (K, m)
                assert abs(a - ao) <= max(1e-10 * max(abs(ao), 1.0),
                                          4 * eps * m / _var_trunc(ao, K)), (K, m, a, ao)
    for xmin in (2, 3, 4):
        lx = math.log(xmin)
        for d in 10 ** rng.uniform(-15, 1.2, 600):
            f, it = C.c_uint32(0), C.c_int(0)
            a = hm.hm_mle_hz_it(lx + d, xmin, C.byref(f), C.byref(it))
            ao, fo = orc.hz_mle(lx + d, xmin)
            io = orc.mle_last_iters()
            assert f.value & 8 == fo & 8, (xmin, d, a, ao)
            if it.value == 200 and io == 200:
                both += 1
                assert fo & 8 == 0, (xmin, d)
                assert abs(a - ao) <= max(1e-10 * ao, 4 * eps * (lx + d) / _var_cut(ao, xmin)), \
                    (xmin, d, a, ao)
    assert both >= 20, both
    for m in 10 ** rng.uniform(-12, math.log10(43.0), 3000):
        f, it = C.c_uint32(0), C.c_int(0)
        a = hm.hm_mle_it(m, C.byref(f), C.byref(it))
        ao, fo = orc.mle(m)
        assert it.value < 200 and orc.mle_last_iters() < 200, m
        assert f.value & 8 == 0 and fo & 8 == 0, m


KH, KGUIDE = 4096, 256 + 52 * 64


def _guide_tables(hm, orc):
    """(label, T) for the guide checks: the library's pure-law tables over the
    exponent range, the truncated law (uniform-like and steep) and the law with
    a lower cutoff (the oracle's tables, which differ from the library's by a
    few ulps at most; any table of increasing values serves)."""
    out = []
    for a in (1.01, 1.05, 1.2, 1.3, 1.4, 1.5, 1.75, 2.0, 2.5, 3.5, 8.0, 20.0, 64.0):
        T = np.zeros(KH)
        hm.hm_table(a, T.ctypes.data_as(C.POINTER(C.c_double)))
        out.append(("pure %g" % a, T))
    for g, K in ((0.25, 1000), (1.0, 4096), (3.0, 20), (-2.0, 4096)):
        T = np.asarray(orc.tz_cdf_table(g, K), np.float64)  # 1..K; T[k] = 1 above K
        out.append(("trunc %g K=%d" % (g, K), np.concatenate([T, np.ones(KH - T.size)])))
    for a, xm in ((1.6, 500), (2.5, 10), (30.0, 3132)):
        out.append(("cutoff %g xmin=%d" % (a, xm), np.asarray(orc.hz_cdf_table(a, xm), np.float64)))
    return out


def test_guide_bounds_and_brackets(hm, orc):
    """The guide the kernels build (guide_refinement, guide_bin_min,
    guide_index: the library's own code compiled for the host) on each table:
    every entry in [1, kH] and non-decreasing; every uniform's bin index
    inside [0, kGuide) (the simulation reads guide[b] and T[g[b] - 1] before
    it knows whether the draw is a tail draw); and for every uniform not in
    the tail, the drawn value min{k : floor(T[k] 2^53) >= m} lies in the
    bracket [g[b], g[b + 1]].  Uniforms: 200,000 random odd m plus every table
    value's integer and its neighbours, and the edges of both guide parts."""
    rng = np.random.default_rng(12)
    for label, T in _guide_tables(hm, orc):
        T = np.ascontiguousarray(T, np.float64)
        assert T.size == KH and np.all(np.diff(T) >= 0), label
        g = np.zeros(KGUIDE + 1, np.uint16)
        sh = hm.hm_guide_build(T.ctypes.data_as(C.POINTER(C.c_double)),
                               g.ctypes.data_as(C.POINTER(C.c_uint16)))
        assert 0 <= sh <= 4 or sh == 8, label
        gi = g.astype(np.int64)
        assert gi.min() >= 1 and gi.max() <= KH and np.all(np.diff(gi) >= 0), label
        TI = (T * 2.0**53).astype(np.uint64)  # floor: T < 1 is exact after scaling
        TI[T >= 1.0] = np.uint64(1 << 53)
        timax = int(TI[-1])
        ms = [rng.integers(1, 1 << 53, 200000, dtype=np.int64).astype(np.uint64) | np.uint64(1)]
        near = (TI.astype(np.int64)[:, None] + np.arange(-2, 3)[None, :]).ravel()
        near = near[(near >= 1) & (near < (1 << 53))].astype(np.uint64) | np.uint64(1)
        # (a uniform's m is odd and below 2^53: timax may be 2^53, T = 1)
        top = (1 << 53) - 1
        edges = np.array([1, 3, (1 << 52) - 1, (1 << 52) + 1, (1 << 53) - 3, top,
                          min(timax, top) | 1, max(min(timax, top) - 2, 1) | 1], np.uint64)
        m = np.concatenate(ms + [near, edges])
        idx = np.zeros(m.size, np.int32)
        hm.hm_guide_index_many(m.ctypes.data_as(C.POINTER(C.c_uint64)), m.size, sh,
                               idx.ctypes.data_as(C.POINTER(C.c_int32)))
        assert idx.min() >= 0 and idx.max() < KGUIDE, label
        lo, hi = gi[idx], gi[idx + 1]
        body = m <= np.uint64(timax)
        x = np.searchsorted(TI, m[body], side="left") + 1
        assert np.all((lo[body] <= x) & (x <= hi[body])), (label, sh)
        # the refinement leaves no uniform of the body in a clamped bin
        if 0 < sh <= 4:
            assert idx[body].max() < KGUIDE - 1, label
        if sh == 8:  # the uniform layout uses bins 0..2047
            assert idx.max() < 2048, label


def test_packed_guide_fast_path(hm, orc):
    """The simulation's one-probe fast path on the packed guide (guide_pack,
    the library's code compiled for the host): x = lo when TI[lo] >= m, else
    the entry's high half, deferred when that is >= kDeferred.  For every
    uniform of the bracket test's sets the result is the drawn value
    min{k : TI[k] >= m} or deferred, and tail uniforms (m > TI[kH]) are always
    deferred; and body uniforms with a bracket one or two values wide are
    deferred only in the bin that straddles TI[kH]."""
    rng = np.random.default_rng(21)
    kdef = 0x8000
    for label, T in _guide_tables(hm, orc):
        T = np.ascontiguousarray(T, np.float64)
        g = np.zeros(KGUIDE + 1, np.uint16)
        sh = hm.hm_guide_build(T.ctypes.data_as(C.POINTER(C.c_double)),
                               g.ctypes.data_as(C.POINTER(C.c_uint16)))
        TI = (T * 2.0**53).astype(np.uint64)
        TI[T >= 1.0] = np.uint64(1 << 53)
        timax = int(TI[-1])
        pk = np.zeros(KGUIDE, np.uint32)
        hm.hm_guide_pack_all(g.ctypes.data_as(C.POINTER(C.c_uint16)), sh, timax,
                             pk.ctypes.data_as(C.POINTER(C.c_uint32)))
        ms = [rng.integers(1, 1 << 53, 100000, dtype=np.int64).astype(np.uint64) | np.uint64(1)]
        near = TI[TI < (1 << 53)].astype(np.int64)
        ms.append((np.concatenate([near - 1, near + 1, near + 3]).clip(1, (1 << 53) - 1)
                   .astype(np.uint64) | np.uint64(1)))
        ms.append(((1 << 53) - rng.integers(1, 1 << 40, 20000, dtype=np.int64))
                  .astype(np.uint64) | np.uint64(1))
        m = np.concatenate(ms)
        idx = np.zeros(m.size, np.int32)
        hm.hm_guide_index_many(m.ctypes.data_as(C.POINTER(C.c_uint64)), m.size, sh,
                               idx.ctypes.data_as(C.POINTER(C.c_int32)))
        e = pk[idx].astype(np.int64)
        lo = e & 0xFFFF
        hiw = e >> 16
        x = np.where(TI[lo - 1] >= m, lo, hiw)
        tail = m > np.uint64(timax)
        assert np.all(x[tail] >= kdef), label
        body = ~tail
        want = np.searchsorted(TI, m[body], side="left") + 1
        xb = x[body]
        ok = xb < kdef
        assert np.array_equal(xb[ok], want[ok]), label
        # narrow brackets defer only in a bin that also holds tail uniforms
        # (the one straddling TI[kH]): a small share of the body
        width = g.astype(np.int64)[idx[body] + 1] - g.astype(np.int64)[idx[body]]
        assert np.mean((width <= 1) & ~ok) < 1e-3, label


def test_guide_refinement_narrows_heavy_tails(hm):
    """The refinement's purpose, on the library's tables: at alpha = 1.2 and
    1.5 the share of body uniforms whose bracket is wider than two values
    (deferred to a search) falls by more than half."""
    rng = np.random.default_rng(3)
    m = rng.integers(1, 1 << 53, 100000, dtype=np.int64).astype(np.uint64) | np.uint64(1)
    for a, sh_expected in ((1.2, 4), (1.5, 3)):
        T = np.zeros(KH)
        hm.hm_table(a, T.ctypes.data_as(C.POINTER(C.c_double)))
        g = np.zeros(KGUIDE + 1, np.uint16)
        sh = hm.hm_guide_build(T.ctypes.data_as(C.POINTER(C.c_double)),
                               g.ctypes.data_as(C.POINTER(C.c_uint16)))
        assert sh == sh_expected
        TI = (T * 2.0**53).astype(np.uint64)
        body = m <= TI[-1]

        def wide(s, gg):
            idx = np.zeros(m.size, np.int32)
            hm.hm_guide_index_many(m.ctypes.data_as(C.POINTER(C.c_uint64)), m.size, s,
                                   idx.ctypes.data_as(C.POINTER(C.c_int32)))
            w = gg.astype(np.int64)[idx + 1] - gg.astype(np.int64)[idx]
            return np.mean(w[body] > 1)
        # the same table's guide without refinement, built in Python
        g0 = np.zeros(KGUIDE + 1, np.int64)
        for b in range(KGUIDE):
            if b < 256:
                mmin = b << 44
            else:
                o, s_ = (b - 256) >> 6, 63 - ((b - 256) & 63)
                N, k = 64 + s_ + 1, o + 6 - 51
                emax = ((N - 1) >> k) if k >= 0 else ((N << (-k)) - 1)
                mmin = (1 << 53) - emax
            j = int(np.searchsorted(TI, np.uint64(mmin), side="left"))
            g0[b] = j + 1 if j < KH else KH
        g0[KGUIDE] = KH
        assert wide(sh, g) < 0.5 * wide(0, g0), a


def test_guide_uniform_layout_for_spread_bounded_support(hm, orc):
    """The truncated law at a small exponent (nearly uniform on 1..K) takes
    the uniform layout, and its share of deferred (wide-bracket) body uniforms
    falls below 1 %, from above half with the log-scale layout; a steep
    truncated law and every pure-law table keep the log-scale layout."""
    rng = np.random.default_rng(4)
    m = rng.integers(1, 1 << 53, 100000, dtype=np.int64).astype(np.uint64) | np.uint64(1)
    for g_, K, uni in ((0.25, 1000, True), (0.5, 1000, True), (3.0, 1000, False)):
        T = np.asarray(orc.tz_cdf_table(g_, K), np.float64)
        T = np.concatenate([T, np.ones(KH - T.size)])
        gg = np.zeros(KGUIDE + 1, np.uint16)
        sh = hm.hm_guide_build(T.ctypes.data_as(C.POINTER(C.c_double)),
                               gg.ctypes.data_as(C.POINTER(C.c_uint16)))
        assert (sh == 8) == uni, (g_, K, sh)
        if uni:
            idx = np.zeros(m.size, np.int32)
            hm.hm_guide_index_many(m.ctypes.data_as(C.POINTER(C.c_uint64)), m.size, sh,
                                   idx.ctypes.data_as(C.POINTER(C.c_int32)))
            w = gg.astype(np.int64)[idx + 1] - gg.astype(np.int64)[idx]
            assert np.mean(w > 1) < 0.01, (g_, K)
    for a in (1.01, 1.2, 2.5, 64.0):
        T = np.zeros(KH)
        hm.hm_table(a, T.ctypes.data_as(C.POINTER(C.c_double)))
        gg = np.zeros(KGUIDE + 1, np.uint16)
        assert hm.hm_guide_build(T.ctypes.data_as(C.POINTER(C.c_double)),
                                 gg.ctypes.data_as(C.POINTER(C.c_uint16))) <= 4
