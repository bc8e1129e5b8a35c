"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks
that each one fails at least one of the pins that the real oracle passes.
This shows the pins constrain every part of the oracle that matters.

Two edits look like mistakes but are not, and are deliberately absent: taking
the KS term at a sample value one-sided (a negative deviation there is always
dominated by the one just below the next sample value, which the other term
covers), and flipping the sign of the Newton derivative (the bracketed
bisection safeguard still converges to the same root)."""
import math
import re
from pathlib import Path

import mpmath as mp
import numpy as np
import pytest

ROOT = Path(__file__).resolve().parent.parent
SRC = ROOT / "oracle" / "zpl_oracle.c"

# (name, original text, planted mistake)
MUTANTS = [
    ("drop EM half term", "z0 += 0.5 * as;", "z0 += 0.0 * as;"),
    ("sign of zeta' integral term", "z1 += a1s * (-L / sm1 - 1.0 / (sm1 * sm1));",
     "z1 += a1s * (L / sm1 - 1.0 / (sm1 * sm1));"),
    ("one Bernoulli term dropped early", "#define ORC_EM_P 10", "#define ORC_EM_P 1"),
    ("CDF index off by one", "T[k - 1] = 1.0 - hurwitz0(alpha, (double)k + 1.0) / z;",
     "T[k - 1] = 1.0 - hurwitz0(alpha, (double)k) / z;"),
    ("uniform without the odd bit", "uint64_t m = (w >> 11) | 1u;", "uint64_t m = (w >> 11);"),
    ("Philox key schedule", "k1 += PHILOX_W1;", "k1 += PHILOX_W0;"),
    ("Philox word order", "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;"),
    ("tail exponent alpha instead of alpha-1",
     "const double beta = alpha - 1.0; /* exact in FP64 for alpha > 1 */",
     "const double beta = alpha; /* planted */"),
    ("tail acceptance skipped", "if (W * gm <= tail_g(beta, (double)X)) return X;", "return X;"),
    ("all-ones rule missing", "s = log(2.0);", "s = 0.0;"),
    ("KS misses the point below each value", "if (d2 > D) D = d2;", "(void)d2;"),
    ("KS against the CDF one value up", "double Fv = 1.0 - hurwitz0(a, (double)v + 1.0) / z;",
     "double Fv = 1.0 - hurwitz0(a, (double)v + 2.0) / z;"),
    ("quantile index off by one", "uint64_t idx = ((uint64_t)R * (uint64_t)num) / (uint64_t)den;",
     "uint64_t idx = ((uint64_t)R * (uint64_t)num) / (uint64_t)den + 1;"),
    ("MLE equation sign", "double g = -r1 - m;", "double g = r1 - m;"),
    ("bootstrap strict inequality", "if (Db[b] >= d) ++ge;", "if (Db[b] > d) ++ge;"),
    # the law with a lower cutoff xmin
    ("xmin draw offset", "return xmin - 1 + (int64_t)lo;", "return xmin + (int64_t)lo;"),
    ("xmin table normalised by zeta(alpha)", "const double z = hurwitz0_rel(alpha, r, r);",
     "const double z = hurwitz0_rel(alpha, 1.0, r);"),
    ("xmin KS normalised by zeta(a)", "const double z = hurwitz0_rel(a, r, r);",
     "const double z = hurwitz0_rel(a, 1.0, r);"),
    ("xmin MLE with zeta(a)", "orc_hurwitz3_scaled(a, q, q, z);",
     "orc_hurwitz3_scaled(a, 1.0, q, z);"),
    ("xmin scaled integral term loses its factor a",
     "const double a1s = r == 1.0 ? pow(a, 1.0 - s) : a * as;",
     "const double a1s = r == 1.0 ? pow(a, 1.0 - s) : as;"),
    ("xmin cutoff rule counts xmin + 2", "tmp[n - 1] = xmin + 1;", "tmp[n - 1] = xmin + 2;"),
    ("xmin scan keeps the largest D", "if (best < 0 || D[c] < D[best]) best = c;",
     "if (best < 0 || D[c] > D[best]) best = c;"),
    ("xmin tail starts at the pure law's", "const double m = (double)(xmin + ORC_TABLE_H);",
     "const double m = (double)(ORC_TABLE_H + 1);"),
    # the truncated law on 1..K
    ("trunc suffix sum one index up", "suf[t] = suf[t + 1] + pow((double)(t + 1), -g);",
     "suf[t] = suf[t + 1] + pow((double)(t + 2), -g);"),
    ("trunc Z' sign", "    z1 -= l * t;", "    z1 += l * t;"),
    ("trunc Z'' without the square", "    z2 += l * l * t;", "    z2 += l * t;"),
    ("trunc table normalised by the wrong sum", "T[k - 1] = 1.0 - suf[k] / suf[0];",
     "T[k - 1] = 1.0 - suf[k] / suf[1];"),
    ("trunc draw never returns 1", "  int lo = 1, hi = K;\n  while (lo < hi) {\n    int mid = lo + (hi - lo) / 2;",
     "  int lo = 2, hi = K;\n  while (lo < hi) {\n    int mid = lo + (hi - lo) / 2;"),
    ("trunc MLE equation sign", "double gval = -r1 - m;", "double gval = r1 - m;"),
    ("trunc NOCONV on rounding noise",
     "if (!(fabs(g_last) <= 0x1p-44 * m)) *flags |= ORC_FLAG_NOCONV;\n  return a;\n}\n\n/* KS distance (eq. 3) of a sorted sample under the truncated law",
     "*flags |= ORC_FLAG_NOCONV;\n  return a;\n}\n\n/* KS distance (eq. 3) of a sorted sample under the truncated law"),
    ("xmin NOCONV on rounding noise",
     "if (!(fabs(g_last) <= 0x1p-44 * m)) *flags |= ORC_FLAG_NOCONV;\n  return a;\n}\n\n/* D over the sorted values",
     "*flags |= ORC_FLAG_NOCONV;\n  return a;\n}\n\n/* D over the sorted values"),
    ("trunc KS below each value at the value", "double Fv1 = 1.0 - suf[v - 1] / z;",
     "double Fv1 = 1.0 - suf[v] / z;"),
    ("trunc KS upper term uses the count below", "double d1 = fabs((double)upto / dn - Fv);",
     "double d1 = fabs((double)below / dn - Fv);"),
    ("trunc all-ones rule missing",
     "    s = log(2.0);\n    *flags |= ORC_FLAG_ALL_ONES;\n  }\n  double a = orc_tz_mle(",
     "    s = 0.0;\n    *flags |= ORC_FLAG_ALL_ONES;\n  }\n  double a = orc_tz_mle("),
]


def _checks(orc):
    """Fast pins; returns the names of those that fail."""
    failed = []
    z2 = orc.zeta3(2.0)
    if abs(z2[0] - math.pi ** 2 / 6) > 1e-15 * 2:
        failed.append("zeta(2)")
    zp2 = float(mp.pi ** 2 / 6 * (mp.euler + mp.log(2 * mp.pi) - 12 * mp.log(mp.glaisher)))
    if abs(z2[1] - zp2) > 1e-14:
        failed.append("zeta'(2)")
    for a in (1.2, 2.5):
        T = orc.cdf_table(a)
        want = 1 - mp.zeta(a, 3) / mp.zeta(a)
        if abs(T[1] - float(want)) > 1e-15:
            failed.append("cdf table")
    if orc.u53(0, 0) != 2.0 ** -53:
        failed.append("u53")
    if list(orc.philox((1, 2, 3, 4), (5, 6))) != [_PHILOX_REF[k] for k in range(4)]:
        failed.append("philox")
    # sampler law: tail fraction and tail mean log at alpha = 1.3
    x, _ = orc.sample(1.3, 40000, 5, 1, 0)
    tail = x[x > 4096].astype(np.float64)
    exp_frac = float(mp.zeta(1.3, 4097) / mp.zeta(1.3))
    if abs(tail.size / x.size - exp_frac) > 6 * math.sqrt(exp_frac / x.size):
        failed.append("tail fraction")
    if tail.size > 50:
        # P(X >= 10 m | X >= m) for m = 4097 under p(k) ~ k^-1.3
        frac10 = np.mean(tail >= 40970)
        want10 = float(mp.zeta(1.3, 40970) / mp.zeta(1.3, 4097))
        if abs(frac10 - want10) > 6 * math.sqrt(want10 * (1 - want10) / tail.size):
            failed.append("tail shape")
    # tail draws whose first proposal the real oracle rejects
    for (a, i), want in _REF["tail"].items():
        if orc.tail_draw(a, 77, 3, 0, i)[0] != want:
            failed.append("tail rejection")
            break
    r = orc.fit(np.ones(10, np.int64))
    if abs(r["D"] - 0.0819313) > 1e-6:
        failed.append("all-ones atom")
    for xs in (np.array([1, 1, 1, 2, 5, 5, 9]), np.array([2, 40, 41, 300])):
        r = orc.fit(xs)
        a = r["alpha_hat"]
        z = mp.zeta(a)
        best, F = mp.mpf(0), mp.mpf(0)
        for t in range(1, int(xs.max()) + 5):
            F += mp.mpf(t) ** (-a) / z
            Sn = mp.mpf(int(np.sum(xs <= t))) / len(xs)
            best = max(best, abs(F - Sn))
        if abs(r["D"] - float(best)) > 1e-12:
            failed.append("KS brute force")
        S = float(np.sum(np.log(xs)))
        if abs(-float(mp.zeta(a, 1, 1) / mp.zeta(a)) - S / len(xs)) > 1e-12:
            failed.append("MLE equation")
    D = np.arange(100, dtype=np.float64)
    if orc.quantile(D, 9, 10) != 90.0:
        failed.append("quantile index")
    ones = orc.bootstrap_pvalue(np.ones(10, np.int64), 300, 3, 1)
    if ones["p_value"] < 0.3:
        failed.append("bootstrap ties")
    failed += _checks_xmin(orc)
    failed += _checks_trunc(orc)
    return failed


def _checks_trunc(orc):
    """Quick pins of the truncated law on 1..K against mpmath sums."""
    failed = []
    K = 20
    with mp.workdps(30):
        for g in (0.0, 1.0, 2.5):
            want = [mp.fsum(mp.mpf(k) ** -g * mp.log(k) ** d for k in range(1, K + 1))
                    for d in range(3)]
            z = orc.tz_norm3(g, K)
            if abs(z[0] - float(want[0])) > 1e-13 * float(want[0]) or \
                    abs(z[1] + float(want[1])) > 1e-13 * float(want[1]) or \
                    abs(z[2] - float(want[2])) > 1e-13 * float(want[2]):
                failed.append("trunc normaliser")
                break
        g = 0.75
        T = orc.tz_cdf_table(g, K)
        Z = mp.fsum(mp.mpf(k) ** -g for k in range(1, K + 1))
        F = [float(mp.fsum(mp.mpf(k) ** -g for k in range(1, t + 1)) / Z) for t in range(1, K + 1)]
    if np.max(np.abs(T - np.array(F))) > 1e-15:
        failed.append("trunc table")
    x = orc.tz_sample(g, K, 200, 5, 3, 11)
    for i in range(200):
        w = orc.philox([i >> 1, 11, 3, 0], [5, 0])
        U = orc.u53(w[2], w[3]) if i & 1 else orc.u53(w[0], w[1])
        if x[i] != 1 + int(np.searchsorted(np.array(F), U, side="left")):
            failed.append("trunc draws")
            break
    xs = np.array([1, 1, 2, 3, 3, 7, 12, 20, 5])
    r = orc.tz_fit(xs, K)
    a = r["alpha_hat"]
    with mp.workdps(30):
        Z = mp.fsum(mp.mpf(k) ** -a for k in range(1, K + 1))
        mu = mp.fsum(mp.log(k) * mp.mpf(k) ** -a for k in range(1, K + 1)) / Z
        best, Fa = mp.mpf(0), mp.mpf(0)
        for t in range(1, K + 1):
            Fa += mp.mpf(t) ** -a / Z
            best = max(best, abs(Fa - mp.mpf(int(np.sum(xs <= t))) / len(xs)))
    if abs(float(mu) - r["S"] / len(xs)) > 1e-12:
        failed.append("trunc MLE equation")
    if abs(r["D"] - float(best)) > 1e-12:
        failed.append("trunc KS")
    # all ones: S := ln 2, and D is the mass above 1 under the fit
    r = orc.tz_fit(np.ones(10, np.int64), K)
    with mp.workdps(30):
        a = mp.findroot(lambda s: mp.fsum(mp.log(k) * mp.mpf(k) ** -s for k in range(1, K + 1))
                        / mp.fsum(mp.mpf(k) ** -s for k in range(1, K + 1)) - mp.log(2) / 10, 4)
        want = 1 - 1 / mp.fsum(mp.mpf(k) ** -a for k in range(1, K + 1))
    if abs(r["D"] - float(want)) > 1e-12:
        failed.append("trunc all-ones atom")
    # K = 2 near the edges: the closed-form root log2((1 - p)/p), m = p ln 2,
    # lies inside [-64, 64], so NOCONV must stay clear
    for e in np.linspace(5, 14, 37):
        for p in (10.0 ** -e, 1 - 10.0 ** -e):
            if orc.tz_mle(math.log(2) * p, 2)[1] & 8:
                failed.append("trunc NOCONV inside the bracket")
                return failed
    return failed


def _checks_xmin(orc):
    """Quick pins of the law with a lower cutoff."""
    failed = []
    # near the edge m -> ln xmin: m above mu(64) (30 digits) has its root
    # below 64, so NOCONV must stay clear
    with mp.workdps(30):
        for xmin in (2, 3):
            w = [(mp.mpf(k) ** -64, mp.log(k)) for k in range(xmin, xmin + 40)]
            mu64 = float(mp.fsum(t * l for t, l in w) / mp.fsum(t for t, _ in w))
            for d in np.geomspace(1e-9, 1e-6, 40):
                m = math.log(xmin) + float(d)
                if m > mu64 * (1 + 1e-14) and orc.hz_mle(m, xmin)[1] & 8:
                    failed.append("xmin NOCONV inside the bracket")
                    break
    T = orc.hz_cdf_table(2.5, 7)
    with mp.workdps(30):
        want = (mp.mpf(7) ** -2.5 + mp.mpf(8) ** -2.5 + mp.mpf(9) ** -2.5) / mp.zeta(2.5, 7)
    if abs(T[2] - float(want)) > 1e-15:
        failed.append("xmin table")
    for a, xmin in ((2.5, 3), (1.6, 500)):
        T = orc.hz_cdf_table(a, xmin)
        x, _ = orc.hz_sample(a, xmin, 300, 9, 2, 11)
        for i in range(300):
            w = orc.philox([i >> 1, 11, 2, 0], [9, 0])
            U = orc.u53(w[2], w[3]) if i & 1 else orc.u53(w[0], w[1])
            body = U <= T[-1]
            if (body and x[i] != xmin + int(np.searchsorted(T, U, side="left"))) or \
                    (not body and x[i] < xmin + 4096):
                failed.append("xmin draws")
                break
    xs = np.array([3, 3, 4, 6, 9, 30, 3, 5])
    r = orc.hz_fit(xs, 3)
    a = r["alpha_hat"]
    with mp.workdps(30):
        z = mp.zeta(a, 3)
        best, F = mp.mpf(0), mp.mpf(0)
        for t in range(3, 40):
            F += mp.mpf(t) ** (-a) / z
            best = max(best, abs(F - mp.mpf(int(np.sum(xs <= t))) / len(xs)))
        mu = -mp.zeta(a, 3, 1) / z
    if abs(r["D"] - float(best)) > 1e-12:
        failed.append("xmin KS")
    if abs(float(mu) - r["S"] / len(xs)) > 1e-12:
        failed.append("xmin MLE equation")
    r = orc.hz_fit(np.full(10, 2), 2)
    if abs(r["S"] - (9 * math.log(2) + math.log(3))) > 1e-12:
        failed.append("xmin cutoff rule")
    # a cutoff of 10^6: q^-s alone underflows there during the iteration
    lx = math.log(10 ** 6)
    a6, f6 = orc.hz_mle(lx + 0.67, 10 ** 6)
    if f6 & orc.FLAG_NOCONV or abs(a6 - 2.4925361995999435) > 1e-12 * a6:
        failed.append("xmin MLE at a large cutoff")
    sc = orc.hz_scan(np.array([1, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89]), [1, 2, 3, 5, 8])
    if sc["best"] != int(np.argmin(sc["D"])):
        failed.append("xmin scan")
    return failed


_PHILOX_REF = {}
_REF = {"tail": {}}


def _reference(orc):
    """Values of the real oracle that the quick pins compare mutants with."""
    if _PHILOX_REF:
        return
    _PHILOX_REF.update(enumerate(orc.philox((1, 2, 3, 4), (5, 6))))
    # draw indices whose first tail proposal is rejected (found with float
    # arithmetic on the oracle's Philox words; the real oracle's answer is
    # the reference)
    key = (77, 0)
    for a in (1.2, 1.5):
        beta, m = a - 1.0, 4097.0
        g = lambda k: 1.0 / (-k * math.expm1(-beta * math.log1p(1.0 / k)))  # noqa: E731
        found = 0
        for i in range(200000):
            w = orc.philox((i, 0, 3, 0x80000000), key)
            V = ((int(w[0]) << 32 | int(w[1])) >> 11 | 1) / 2.0 ** 53
            W = ((int(w[2]) << 32 | int(w[3])) >> 11 | 1) / 2.0 ** 53
            Y = m * V ** (-1.0 / beta)
            if Y >= 2.0 ** 62:
                continue
            if W * g(m) > g(math.floor(Y)):
                _REF["tail"][(a, i)] = orc.tail_draw(a, 77, 3, 0, i)[0]
                found += 1
                if found == 3:
                    break
    assert len(_REF["tail"]) >= 4


def test_real_oracle_passes_the_quick_pins(orc):
    _reference(orc)
    assert _checks(orc) == []


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(orc, tmp_path, name, orig, planted):
    _reference(orc)
    src = SRC.read_text()
    assert src.count(orig) >= 1, "mutation site not found: %s" % name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(orig, planted, 1))
    lib = orc.compile_variant(mutant, tmp_path / ("m_%s.so" % re.sub(r"\W+", "_", name)))
    with orc.use_library(lib):
        failed = _checks(orc)
    assert failed, "planted mistake '%s' passed every pin" % name
