// zpl_math.hpp -- scalar arithmetic of the Zipf/KS Monte Carlo path.
//
// Everything here is plain scalar FP64/integer code marked __host__ __device__
// so that one definition serves every GPU kernel (lane, wave and heavy paths
// and the dataset fit), and can also be compiled for the host to test its
// logic on a CPU.  The library is built with -ffp-contract=off: every fused
// multiply-add is an explicit fma(), so a given input produces the same bits
// in whichever kernel the function is inlined.  That is what makes a replicate
// give bit-identical (alpha_hat, D) in every execution mode, and makes ties
// between a bootstrap replicate and the observed statistic exact.
//
// Reference: E. Rappos and S. Robert, "Using GPU Simulation to Accurately Fit
// to the Power-Law Distribution" (2013).  Eq. (1): p(k) = k^-a / zeta(a);
// eq. (2): zeta'(a)/zeta(a) = -(1/N) sum ln x_i; eq. (3): K = sup|F* - S|.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zpl_exp2_table.hpp"
#include "zpl_kernels.hpp"

#define ZPL_HD __host__ __device__ __forceinline__

namespace zpl {

// CDF table length: values 1..kH are drawn by table search, larger ones by
// the rejection tail.  Part of the sampling contract (samples depend on it).
constexpr int kH = 4096;
// First value of the tail.
constexpr double kTailM = 4097.0;
// Philox counter word 3 for tail proposals: kTailDomain | attempt.
constexpr uint32_t kTailDomain = 0x80000000u;

constexpr uint32_t kFlagAllOnes = 1u;
constexpr uint32_t kFlagTailCapped = 2u;
constexpr uint32_t kFlagBisect = 4u;
constexpr uint32_t kFlagNoConv = 8u;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies counter words 0 and 2 by the two round constants (32x32->64),
// mixes the high halves with words 1, 3 and the key, and the key is bumped by
// the two Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c: one three-input bitwise instruction on gfx950.
ZPL_HD uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

ZPL_HD Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

// Odd multiple of 2^-53 in (0,1) from the 64-bit word hi:lo.
ZPL_HD double u53(uint32_t hi, uint32_t lo) {
  const uint64_t m = ((((uint64_t)hi) << 32 | (uint64_t)lo) >> 11) | 1ull;
  return (double)m * 0x1p-53;
}

// splitmix64's output finaliser; summed over draws it is a fingerprint of the
// multiset of drawn values (used only to check histograms bit for bit).
ZPL_HD uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Hurwitz zeta by Euler-Maclaurin with no direct terms, valid for q >= 17:
//   zeta(s,q) = q^-s [ q/(s-1) + 1/2 + sum_{i=1..8} c_i (s)_{2i-1} q^-(2i-1) ]
// with c_i = B_2i/(2i)! and (s)_m the rising factorial.  The factors that
// depend on s alone, k_i = c_i (s)_{2i-1} and 1/(s-1), are computed once per
// exponent (EmCoef); the series is then a polynomial in 1/q^2 evaluated
// innermost-first (smallest terms first).
// ---------------------------------------------------------------------------
struct EmCoef {
  double s, ism1, k[8];
};

ZPL_HD EmCoef em_coef(double s) {
  const double c[8] = {1.0 / 12.0,         -1.0 / 720.0,
                       1.0 / 30240.0,      -1.0 / 1209600.0,
                       1.0 / 47900160.0,   -691.0 / 1307674368000.0,
                       1.0 / 74724249600.0, -3617.0 / 10670622842880000.0};
  EmCoef e;
  e.s = s;
  e.ism1 = 1.0 / (s - 1.0);
  double P = s;  // (s)_{2i-1}
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    e.k[i] = c[i] * P;
    P *= (s + (double)(2 * i + 1)) * (s + (double)(2 * i + 2));
  }
  return e;
}

// 1/x to about one ulp: the hardware reciprocal refined by two Newton steps.
ZPL_HD double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}

// q^-s = exp(-s ln q) with the product s ln q kept exact (p + e), so the
// product's rounding (up to s ln q ulps of relative error) is not amplified.
ZPL_HD double pow_neg(double s, double lnq) {
  const double p = s * lnq;
  const double e = fma(s, lnq, -p);
  const double r = exp(-p);
  return fma(-e, r, r);
}

// zeta(s, q) for q >= 17; lnq = ln q.
ZPL_HD double hurwitz_tail(const EmCoef& E, double q, double lnq) {
  const double qs = pow_neg(E.s, lnq);
  const double iq = recip(q), iq2 = iq * iq;
  double acc = E.k[7];
#pragma unroll
  for (int i = 6; i >= 0; --i) acc = fma(acc, iq2, E.k[i]);
  return qs * (fma(q, E.ism1, 0.5) + acc * iq);
}

// Reciprocal for the s-derivative factors of the Euler-Maclaurin corrections
// at q = 17.  The hardware reciprocal is accurate to about 2^-24 (measured on
// gfx950); at q = 17 that moves alpha_hat by at most about 3e-13 relative
// (the error injected into a host build), so it suffices there.  The law with
// a lower cutoff uses recip instead: with a large xmin the variance of ln X
// is small and eq. (2) amplifies errors in zeta'/zeta.
ZPL_HD double rcp_corr(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(x);
#else
  return 1.0 / x;
#endif
}

// k^-s for k = 2..16 from the six prime powers 2,3,5,7,11,13 (one exp each)
// multiplied in a fixed order.  pw[k] for k = 0..16 (pw[0], pw[1] unused).
ZPL_HD void small_powers(double s, const double* __restrict__ ln, double pw[17]) {
  const double p2 = pow_neg(s, ln[2]), p3 = pow_neg(s, ln[3]), p5 = pow_neg(s, ln[5]),
               p7 = pow_neg(s, ln[7]), p11 = pow_neg(s, ln[11]), p13 = pow_neg(s, ln[13]);
  const double p4 = p2 * p2, p8 = p4 * p2;
  pw[0] = 0.0;
  pw[1] = 1.0;
  pw[2] = p2;
  pw[3] = p3;
  pw[4] = p4;
  pw[5] = p5;
  pw[6] = p2 * p3;
  pw[7] = p7;
  pw[8] = p8;
  pw[9] = p3 * p3;
  pw[10] = p2 * p5;
  pw[11] = p11;
  pw[12] = p4 * p3;
  pw[13] = p13;
  pw[14] = p2 * p7;
  pw[15] = p3 * p5;
  pw[16] = p4 * p4;
}

// zeta(s), zeta'(s), zeta''(s): direct terms k = 1..16 (ln k from `ln`, the
// library's table of natural logs) plus the Euler-Maclaurin tail at 17 and
// its first two s-derivatives.  Summed smallest-first in a fixed order.
struct Z3 {
  double z0, z1, z2;
};

ZPL_HD Z3 zeta3(double s, const double* __restrict__ ln) {
  const double q = 17.0;
  const double L = ln[17];
  const double iq = 1.0 / q, iq2 = iq * iq;
  // Q(s) = q/(s-1) + 1/2 + sum_i c_i P_i(s) q^-(2i-1), P_i = (s)_{2i-1};
  // Q' and Q'' use P' = P sum 1/(s+k) and P'' = P ((sum 1/(s+k))^2 - sum 1/(s+k)^2).
  const double c[8] = {1.0 / 12.0,         -1.0 / 720.0,
                       1.0 / 30240.0,      -1.0 / 1209600.0,
                       1.0 / 47900160.0,   -691.0 / 1307674368000.0,
                       1.0 / 74724249600.0, -3617.0 / 10670622842880000.0};
  const double is = rcp_corr(s);
  double P = s, sg1 = is, sg2 = is * is, E = iq;
  double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double ce = c[i] * E;
    Q0 = fma(ce, P, Q0);
    Q1 = fma(ce, P * sg1, Q1);
    Q2 = fma(ce, P * fma(sg1, sg1, -sg2), Q2);
    const double u = s + (double)(2 * i + 1), v = s + (double)(2 * i + 2);
    const double iu = rcp_corr(u), iv = rcp_corr(v);
    P *= u * v;
    sg1 += iu + iv;
    sg2 += iu * iu + iv * iv;
    E *= iq2;
  }
  const double sm1 = s - 1.0, ism1 = 1.0 / sm1;
  Q0 += 0.5;
  Q0 += q * ism1;
  Q1 += -q * ism1 * ism1;
  Q2 += 2.0 * q * ism1 * ism1 * ism1;
  const double qs = pow_neg(s, L);
  // d/ds [q^-s Q] = q^-s (Q' - L Q); d2/ds2 = q^-s (Q'' - 2 L Q' + L^2 Q)
  double z0 = qs * Q0;
  double z1 = qs * fma(-L, Q0, Q1);
  double z2 = qs * fma(L * L, Q0, fma(-2.0 * L, Q1, Q2));
  double pw[17];
  small_powers(s, ln, pw);
#pragma unroll
  for (int k = 16; k >= 2; --k) {
    const double lk = ln[k];
    const double t = pw[k];
    z0 += t;
    z1 = fma(-lk, t, z1);
    z2 = fma(lk * lk, t, z2);
  }
  z0 += 1.0;
  return Z3{z0, z1, z2};
}

// ---------------------------------------------------------------------------
// MLE, eq. (2): solve mu(a) := -zeta'(a)/zeta(a) = m, m = S/n.  mu decreases
// strictly (mu' = -Var[ln X]), so the root is unique.  Newton-Raphson is run
// on ln mu(a) - ln m (nearly linear in a for large a), inside a bracket
// [1 + 2^-20, 64] that shrinks with the sign of mu - m; a step leaving the
// bracket becomes a bisection.  Stops once |step| <= 2^-40 a: convergence is
// quadratic, so the iterate after such a step is at the FP64 noise level of
// mu (a tighter test would only chase that noise).  The rule shared by the
// three laws' solvers: at most kMleCap iterations, and at the cap kFlagNoConv
// only when the last residual |mu - m| exceeds 2^-44 m (the rounding noise
// of an FP64 mu), so the flag means that no root was found.  `iters`, when
// given, receives the iteration count (host checks only).
// ---------------------------------------------------------------------------
constexpr int kMleCap = 200;

ZPL_HD double mle_alpha(double m, const double* __restrict__ ln, uint32_t* flags,
                        int* iters = nullptr) {
  double lo = 1.0 + 0x1p-20, hi = 64.0;
  // initial guess: mu ~ 1/(a-1) - gamma near a = 1; mu ~ ln2 2^-a for large a
  double a1 = 1.0 + 1.0 / (m + 0.5772156649015329);
  double a2 = log2(ln[2] / m);
  double a = a1 > a2 ? a1 : a2;
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  const double lm = log(m);
  double gl = 0.0;  // the last residual of eq. 2
  int it = 0;
  for (; it < kMleCap; ++it) {
    const Z3 z = zeta3(a, ln);
    const double mu = -z.z1 / z.z0;
    if (mu == m) break;
    gl = mu - m;
    if (mu > m)
      lo = a;
    else
      hi = a;
    const double var = fma(-mu, mu, z.z2 / z.z0);
    double an = a + (log(mu) - lm) * (mu / var);
    // the bracket is closed: a converged step may land exactly on lo or hi
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= kFlagBisect;
    }
    const bool done = fabs(an - a) <= 0x1p-40 * a;
    a = an;
    if (done) break;
  }
  if (iters) *iters = it < kMleCap ? it + 1 : it;
  if (it == kMleCap && !(fabs(gl) <= 0x1p-44 * m)) *flags |= kFlagNoConv;
  return a;
}

// ln of an integer value: from the table for v <= kH + 1, else computed.
ZPL_HD double ln_value(int64_t v, const double* __restrict__ ln) {
  return v <= (int64_t)(kH + 1) ? ln[v] : log((double)v);
}

// ---------------------------------------------------------------------------
// zeta(s, q) for the law with a lower cutoff, where it is the whole
// normaliser rather than a small tail of zeta(s).  The Euler-Maclaurin terms
// shrink like ((s + 2i) / (2 pi q))^2: with eight Bernoulli terms the
// remainder is below 1e-16 relative from q = 1.5 s + 10 on (s <= 64, checked
// against partial sums at 40 digits), while at q = 17 it reaches 4e-15 at
// s = 10 and 2e-4 at s = 64.  So the tail starts at q0 = em_start(s) =
// ceil(1.6 s + 10) (a margin over 1.5 s + 10; 17 for s <= 4.375, where
// nothing changes) and the terms below it are summed directly.
// ---------------------------------------------------------------------------
ZPL_HD int64_t em_start(double s) {
  const double q = ceil(fma(1.6, s, 10.0));
  return q > 17.0 ? (int64_t)q : 17;
}

// Where zeta(s, q) itself (q >= 2) starts its Euler-Maclaurin tail:
// em_start(s), or 2q if that is smaller (the tail from 2q on weighs about
// 2^(1-s) of zeta(s, q) when em_start(s) > 2q, which outweighs its larger
// Euler-Maclaurin error: the product stays below 1e-18), and at least 17.
ZPL_HD int64_t em_point(double s, int64_t q) {
  const int64_t e = em_start(s);
  const int64_t t = q < (e + 1) / 2 ? 2 * q : e;  // no 2q overflow for large q
  return t > 17 ? t : 17;
}

// ---------------------------------------------------------------------------
// The law with a lower cutoff xmin (p(k) = k^-a / zeta(a, xmin), k >= xmin;
// the practice the paper cites for fitting, xmin = 1 being its own case).
// zeta(s, xmin) and its first two s-derivatives: direct terms k = xmin..q-1
// (none when xmin >= q), largest k first, after the Euler-Maclaurin tail at
// q = max(xmin, em_point(s, xmin)) and its derivatives (em_point keeps that
// tail accurate at large s; it is 17 for s <= 4.375, as zeta3 uses for
// xmin = 1).  All three are returned multiplied by xmin^s: every power is
// taken as (k/xmin)^-s, the logarithms the derivatives bring down stay ln k.
// The factor cancels in mu = -z1/z0 and in the variance, and without it k^-s
// underflows for s ln k > 708 (at s = 64 from k of about 6.5e4).
// ---------------------------------------------------------------------------
ZPL_HD Z3 hurwitz3(double s, int64_t xmin, const double* __restrict__ ln) {
  const int64_t q0 = em_point(s, xmin);
  const int64_t qi = xmin < q0 ? q0 : xmin;
  const double q = (double)qi;
  const double L = ln_value(qi, ln);
  const double ix = 1.0 / (double)xmin;
  const double iq = 1.0 / q, iq2 = iq * iq;
  const double c[8] = {1.0 / 12.0,         -1.0 / 720.0,
                       1.0 / 30240.0,      -1.0 / 1209600.0,
                       1.0 / 47900160.0,   -691.0 / 1307674368000.0,
                       1.0 / 74724249600.0, -3617.0 / 10670622842880000.0};
  // full-precision reciprocals: with a large cutoff the variance of ln X is
  // small and eq. (2) amplifies any error in zeta'/zeta
  const double is = recip(s);
  double P = s, sg1 = is, sg2 = is * is, E = iq;
  double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double ce = c[i] * E;
    Q0 = fma(ce, P, Q0);
    Q1 = fma(ce, P * sg1, Q1);
    Q2 = fma(ce, P * fma(sg1, sg1, -sg2), Q2);
    const double u = s + (double)(2 * i + 1), v = s + (double)(2 * i + 2);
    const double iu = recip(u), iv = recip(v);
    P *= u * v;
    sg1 += iu + iv;
    sg2 += iu * iu + iv * iv;
    E *= iq2;
  }
  const double sm1 = s - 1.0, ism1 = 1.0 / sm1;
  Q0 += 0.5;
  Q0 += q * ism1;
  Q1 += -q * ism1 * ism1;
  Q2 += 2.0 * q * ism1 * ism1 * ism1;
  // powers relative to xmin: (k/xmin)^-s with ln(k/xmin) = log1p((k - xmin)/xmin)
  const double qs = qi == xmin ? 1.0 : pow_neg(s, log1p((double)(qi - xmin) * ix));
  double z0 = qs * Q0;
  double z1 = qs * fma(-L, Q0, Q1);
  double z2 = qs * fma(L * L, Q0, fma(-2.0 * L, Q1, Q2));
  for (int64_t k = qi - 1; k >= xmin; --k) {
    const double lk = ln[k];
    const double t = k == xmin ? 1.0 : pow_neg(s, log1p((double)(k - xmin) * ix));
    z0 += t;
    z1 = fma(-lk, t, z1);
    z2 = fma(lk * lk, t, z2);
  }
  return Z3{z0, z1, z2};
}

// MLE of eq. (2) with the Hurwitz zeta: mu(a) = -zeta'(a,xmin)/zeta(a,xmin)
// = E_a[ln X] decreases from +inf (a -> 1) to ln xmin (a -> inf).  Newton on
// mu(a) - m in the bracket [1 + 2^-20, 64] with a bisection safeguard, from
// the continuous-Pareto guess a = 1 + 1/(m - ln(xmin - 1/2)); stops after a
// step of at most 2^-40 a.  A root above 64 (m <= mu(64), a sample close to
// a large cutoff) gives 64 with kFlagNoConv.  xmin >= 2.
ZPL_HD double mle_alpha_hz(double m, int64_t xmin, const double* __restrict__ ln,
                           uint32_t* flags, int* iters = nullptr) {
  if (iters) *iters = 0;
  double lo = 1.0 + 0x1p-20, hi = 64.0;
  {
    const Z3 z = hurwitz3(hi, xmin, ln);
    if (!(m > -z.z1 / z.z0)) {
      *flags |= kFlagNoConv;
      return hi;
    }
  }
  double a = 1.0 + 1.0 / (m - log((double)xmin - 0.5));
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  double gl = 0.0;  // the last residual of eq. 2
  for (int it = 0; it < kMleCap; ++it) {
    if (iters) *iters = it + 1;
    const Z3 z = hurwitz3(a, xmin, ln);
    const double r1 = z.z1 / z.z0;
    const double g = -r1 - m;
    if (g == 0.0) return a;
    gl = g;
    if (g > 0.0)
      lo = a;
    else
      hi = a;
    const double gp = -fma(-r1, r1, z.z2 / z.z0);
    double an = a - g / gp;
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= kFlagBisect;
    }
    if (fabs(an - a) <= 0x1p-40 * a) return an;
    a = an;
  }
  // Near the edge m -> ln xmin eq. 2 fixes the root only to about
  // eps m / Var(ln X), coarser than the step test: a residual within the
  // rounding noise of mu is a root as far as FP64 can tell, not a failure.
  if (!(fabs(gl) <= 0x1p-44 * m)) *flags |= kFlagNoConv;
  return a;
}

// ---------------------------------------------------------------------------
// Truncated law on 1..K (Sect. 1 with a finite upper limit): Z_K(s) =
// sum_{k<=K} k^-s and its first two s-derivatives by direct summation, index
// K down to 1.  Defined for every real s; |s| <= 64 and K <= 4097 keep every
// term below 2^768.
// ---------------------------------------------------------------------------
ZPL_HD Z3 zeta3_trunc(double s, uint32_t K, const double* __restrict__ ln) {
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  for (int k = (int)K; k >= 2; --k) {
    const double l = ln[k];
    const double t = pow_neg(s, l);
    z0 += t;
    z1 = fma(-l, t, z1);
    z2 = fma(l * l, t, z2);
  }
  z0 += 1.0;
  return Z3{z0, z1, z2};
}

// M_k(z) = int_0^1 v^k e^(z v) dv for k = 0, 1, 2: the power series
// sum_m z^m / (m! (m + k + 1)) for |z| <= 2 (32 terms by Horner's rule; the
// last is below 2^-80 of the sum), else the closed forms
// M_0 = (e^z - 1)/z, M_1 = (e^z (z - 1) + 1)/z^2, M_2 = (e^z (z^2 - 2z + 2) - 2)/z^3
// (the largest cancellation there, at z = -2, costs under two bits).
struct MomentCoef {
  double c[3][32];  // 1 / (m! (m + k + 1))
};
constexpr MomentCoef moment_coef() {
  MomentCoef t{};
  double f = 1.0;  // m!
  for (int m = 0; m < 32; ++m) {
    if (m > 0) f *= (double)m;
    for (int k = 0; k < 3; ++k) t.c[k][m] = 1.0 / (f * (double)(m + k + 1));
  }
  return t;
}

ZPL_HD void moments012(double z, double& m0, double& m1, double& m2) {
  if (fabs(z) <= 2.0) {
    constexpr MomentCoef C = moment_coef();
    double a0 = C.c[0][31], a1 = C.c[1][31], a2 = C.c[2][31];
#pragma unroll
    for (int m = 30; m >= 0; --m) {
      a0 = fma(a0, z, C.c[0][m]);
      a1 = fma(a1, z, C.c[1][m]);
      a2 = fma(a2, z, C.c[2][m]);
    }
    m0 = a0;
    m1 = a1;
    m2 = a2;
    return;
  }
  const double ez = exp(z), iz = 1.0 / z;
  m0 = expm1(z) * iz;
  m1 = fma(ez, z - 1.0, 1.0) * iz * iz;
  m2 = fma(ez, fma(z, z - 2.0, 2.0), -2.0) * iz * iz * iz;
}

// Z_K(s) and its first two s-derivatives with Euler-Maclaurin summation of
// the terms k = q0..K, for every real s (the truncated law allows s <= 1):
// sum_{k=q0..K} k^-s = I + (q0^-s + K^-s)/2
//                      + sum_i c_i (s)_{2i-1} (q0^(-s-2i+1) - K^(-s-2i+1)),
// I = int_{q0}^{K} x^-s dx = q0^(1-s) D M_0(u D) with u = 1 - s, D = ln(K/q0)
// (and I' = -q0^(1-s) (ln q0 D M_0 + D^2 M_1), I'' = q0^(1-s) (ln^2 q0 D M_0
// + 2 ln q0 D^2 M_1 + D^3 M_2), the moments M_k of moments012, which keep
// s = 1 regular), the rising factorials and their derivatives by the
// product rule (no division by s + j, which vanishes at negative integers).
// q0 = em_start(|s|) (17 up to |s| = 4.375) keeps eight Bernoulli terms
// below 1e-16 relative, as for the Hurwitz zeta; k = 1..q0-1 are summed
// directly.  Used once K is 48 or more above q0, where it is cheaper than the
// K direct terms (a few exps against K).
// Out of line: it is long, and inlined into every finish it would crowd the
// registers of the draw loops around them.
__host__ __device__ __noinline__ static Z3 zeta3_trunc_em(double s, uint32_t K,
                                                          const double* __restrict__ ln) {
  const int64_t q0 = em_start(fabs(s));
  const double c[8] = {1.0 / 12.0,         -1.0 / 720.0,
                       1.0 / 30240.0,      -1.0 / 1209600.0,
                       1.0 / 47900160.0,   -691.0 / 1307674368000.0,
                       1.0 / 74724249600.0, -3617.0 / 10670622842880000.0};
  const double qa = (double)q0, qb = (double)K;
  const double la = ln[q0], lb = ln[K];
  const double fa = pow_neg(s, la), fb = pow_neg(s, lb);  // q0^-s, K^-s
  const double ia2 = 1.0 / (qa * qa), ib2 = 1.0 / (qb * qb);
  // Bernoulli terms: (s)_{2i-1} and its s-derivatives P1, P2
  double P = s, P1 = 1.0, P2 = 0.0;
  double Ea = fa / qa, Eb = fb / qb;  // q^(-s-2i+1)
  double b0 = 0.0, b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // value c P (Ea - Eb); d/ds: c (P1 (Ea - Eb) - P (la Ea - lb Eb));
    // d2/ds2: c (P2 (Ea - Eb) - 2 P1 (la Ea - lb Eb) + P (la^2 Ea - lb^2 Eb))
    const double d0 = Ea - Eb;
    const double d1 = fma(la, Ea, -lb * Eb);
    const double d2 = fma(la * la, Ea, -(lb * lb) * Eb);
    b0 = fma(c[i], P * d0, b0);
    b1 = fma(c[i], fma(P1, d0, -P * d1), b1);
    b2 = fma(c[i], fma(P2, d0, fma(-2.0 * P1, d1, P * d2)), b2);
#pragma unroll
    for (int j = 1; j <= 2; ++j) {  // times (s + 2i + j - ... ): two more factors
      const double f = s + (double)(2 * i + j);
      P2 = fma(P2, f, 2.0 * P1);
      P1 = fma(P1, f, P);
      P *= f;
    }
    Ea *= ia2;
    Eb *= ib2;
  }
  // the integral
  const double D = lb - la;
  double m0, m1, m2;
  moments012((1.0 - s) * D, m0, m1, m2);
  const double g = fa * qa;  // q0^(1-s)
  const double i0 = g * D * m0;
  const double i1 = -g * fma(la * D, m0, D * D * m1);
  const double i2 = g * fma(la * la * D, m0, fma(2.0 * la * D * D, m1, D * D * D * m2));
  // the end terms (f(q0) + f(K))/2
  double z0 = i0 + 0.5 * (fa + fb) + b0;
  double z1 = i1 - 0.5 * fma(la, fa, lb * fb) + b1;
  double z2 = i2 + 0.5 * fma(la * la, fa, (lb * lb) * fb) + b2;
  // direct terms q0-1 down to 2, then 1
  if (q0 == 17) {
    double pw[17];
    small_powers(s, ln, pw);
#pragma unroll
    for (int k = 16; k >= 2; --k) {
      const double lk = ln[k];
      const double t = pw[k];
      z0 += t;
      z1 = fma(-lk, t, z1);
      z2 = fma(lk * lk, t, z2);
    }
  } else {
    for (int k = (int)q0 - 1; k >= 2; --k) {
      const double lk = ln[k];
      const double t = pow_neg(s, lk);
      z0 += t;
      z1 = fma(-lk, t, z1);
      z2 = fma(lk * lk, t, z2);
    }
  }
  z0 += 1.0;
  return Z3{z0, z1, z2};
}

// The truncated law's sums: Euler-Maclaurin once K is 48 or more above the
// direct range, else the K direct terms.
ZPL_HD Z3 zeta3_trunc_fast(double s, uint32_t K, const double* __restrict__ ln) {
  if ((int64_t)K >= em_start(fabs(s)) + 48) return zeta3_trunc_em(s, K, ln);
  return zeta3_trunc(s, K, ln);
}

// MLE of eq. (2) with the finite sums: mu(s) = -Z_K'/Z_K decreases strictly
// from ln K (s -> -inf) to 0 (s -> +inf).  The same safeguarded Newton
// iteration as mle_alpha on [-64, 64]; an iterate ending at the bracket edge
// is checked against mu at the edge, and when m has no root inside the
// bracket the edge is returned with kFlagNoConv.
ZPL_HD double mle_alpha_trunc(double m, uint32_t K, const double* __restrict__ ln,
                              uint32_t* flags, int* iters = nullptr) {
  double lo = -64.0, hi = 64.0;
  double a1 = 1.0 + 1.0 / (m + 0.5772156649015329);
  double a2 = log2(ln[2] / m);
  double a = a1 > a2 ? a1 : a2;
  if (!(a > lo && a < hi)) a = 0.0;
  const double lm = log(m);
  double gl = 0.0;  // the last residual of eq. 2
  int it = 0;
  for (; it < kMleCap; ++it) {
    const Z3 z = zeta3_trunc_fast(a, K, ln);
    const double mu = -z.z1 / z.z0;
    if (mu == m) break;
    gl = mu - m;
    if (mu > m)
      lo = a;
    else
      hi = a;
    const double var = fma(-mu, mu, z.z2 / z.z0);
    double an = a + (log(mu) - lm) * (mu / var);
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= kFlagBisect;
    }
    const double scale = fabs(a) > 1.0 ? fabs(a) : 1.0;
    const bool done = fabs(an - a) <= 0x1p-40 * scale;
    a = an;
    if (done) break;
  }
  // a residual within the rounding noise of mu is a root to FP64 precision
  // (near the edges the step test is out of reach), as for mle_alpha_hz
  if (iters) *iters = it < kMleCap ? it + 1 : it;
  if (it == kMleCap && !(fabs(gl) <= 0x1p-44 * m)) *flags |= kFlagNoConv;
  // Near an edge, is the root inside the bracket?  mu tends to ln K as s
  // falls, and for small K it reaches ln K to FP64 rounding well inside the
  // bracket (K = 2: from s of about -53 on), where an iterate can stop with
  // mu == m although m (every value equal to K) has no root: check the lower
  // edge then too.
  if (fabs(a) > 63.0 || (a < 0.0 && m >= ln[K] * (1.0 - 0x1p-50))) {
    const double e = a > 0.0 ? 64.0 : -64.0;
    const Z3 z = zeta3_trunc_fast(e, K, ln);
    const double mue = -z.z1 / z.z0;
    if (a > 0.0 ? !(m > mue) : !(m < mue)) {
      *flags |= kFlagNoConv;
      return e;
    }
  }
  return a;
}

// ---------------------------------------------------------------------------
// Unnormalised survival zeta(a, t+1) = sum_{k > t} k^-a, so that
// F(t; a) = 1 - zeta(a,t+1)/zeta(a) (eq. 1 summed).  suf[t], t = 0..16, holds
// it for small t (suf[0] = zeta(a)); larger t use hurwitz_tail.
// ---------------------------------------------------------------------------
ZPL_HD void survival_head(const EmCoef& E, const double* __restrict__ ln, double suf[17]) {
  double pw[17];
  small_powers(E.s, ln, pw);
  suf[16] = hurwitz_tail(E, 17.0, ln[17]);
#pragma unroll
  for (int t = 15; t >= 1; --t) suf[t] = suf[t + 1] + pw[t + 1];
  suf[0] = suf[1] + 1.0;
}

ZPL_HD void survival_head(double a, const double* __restrict__ ln, double suf[17]) {
  survival_head(em_coef(a), ln, suf);
}

// zeta(a, v+1) for an integer 16 <= v < 2^63 (v + 1 may not fit in int64).
ZPL_HD double survival_next(const EmCoef& E, int64_t v, const double* __restrict__ ln) {
  if (v < (int64_t)kH + 1) return hurwitz_tail(E, (double)(v + 1), ln[v + 1]);
  const double q = (double)v + 1.0;
  return hurwitz_tail(E, q, log(q));
}

ZPL_HD double survival_next(double a, int64_t v, const double* __restrict__ ln) {
  return survival_next(em_coef(a), v, ln);
}

// The direct part of survival_next_cut: zeta(s, v+1) as the tail at q0 plus
// the terms v+1..q0-1, largest first (k < q0 <= 113: from the ln table).
// Out of line: only large exponents take it, and inlined it would crowd the
// registers of the KS loops that call it.
static __host__ __device__ __noinline__ double survival_cut_direct(double s, int64_t v, int64_t q0,
                                                                   const double* __restrict__ ln) {
  double z = hurwitz_tail(em_coef(s), (double)q0, ln[q0]);
  for (int64_t k = q0 - 1; k > v; --k) z += pow_neg(s, ln[k]);
  return z;
}

// zeta(a, v+1) for an integer 16 <= v < 2^63, accurate at any a <= 64: the
// Euler-Maclaurin tail at max(v + 1, em_point(a, v + 1)), then the direct
// terms below it.
ZPL_HD double survival_next_cut(const EmCoef& E, int64_t v, const double* __restrict__ ln) {
  if (v >= em_start(E.s) - 1) return survival_next(E, v, ln);  // (v + 1 may not fit)
  const int64_t q0 = em_point(E.s, v + 1);
  if (v >= q0 - 1) return survival_next(E, v, ln);
  return survival_cut_direct(E.s, v, q0, ln);
}

// zeta(a, v+1) xmin^a for the law with a cutoff xmin >= 17 and v >= xmin - 1:
// as survival_next_cut, with every power relative to xmin,
// (k/xmin)^-a = exp(-a log1p((k - xmin)/xmin)), so that it stays representable
// however large xmin^-a is (ratios of these give the CDF; the factor cancels).
__host__ __device__ __noinline__ static double survival_rel_direct(double s, int64_t v, int64_t q0,
                                                                   int64_t xmin) {
  const double ix = 1.0 / (double)xmin;
  double z = hurwitz_tail(em_coef(s), (double)q0, log1p((double)(q0 - xmin) * ix));
  for (int64_t k = q0 - 1; k > v; --k)
    z += k == xmin ? 1.0 : pow_neg(s, log1p((double)(k - xmin) * ix));
  return z;
}

// hurwitz_tail takes the logarithm only for its power q^-a, so handing it
// ln(q/xmin) gives the tail relative to xmin^-a.
ZPL_HD double survival_rel(const EmCoef& E, int64_t v, int64_t xmin) {
  if (v < em_start(E.s) - 1) {  // direct terms below the tail, as survival_next_cut
    const int64_t q0 = em_point(E.s, v + 1);
    if (v < q0 - 1) return survival_rel_direct(E.s, v, q0, xmin);
  }
  const double lrel = v + 1 == xmin ? 0.0 : log1p((double)(v + 1 - xmin) / (double)xmin);
  return hurwitz_tail(E, (double)v + 1.0, lrel);
}

// (v/xmin)^-a for v >= xmin: one term of survival_rel.
ZPL_HD double pow_rel(double a, int64_t v, int64_t xmin) {
  return v == xmin ? 1.0 : pow_neg(a, log1p((double)(v - xmin) / (double)xmin));
}

// survival_head with an accurate suf[16] = zeta(a, 17) (see em_start).
ZPL_HD void survival_head_cut(const EmCoef& E, const double* __restrict__ ln, double suf[17]) {
  double pw[17];
  small_powers(E.s, ln, pw);
  suf[16] = survival_next_cut(E, 16, ln);
#pragma unroll
  for (int t = 15; t >= 1; --t) suf[t] = suf[t + 1] + pw[t + 1];
  suf[0] = suf[1] + 1.0;
}

// ---------------------------------------------------------------------------
// Exact accumulation of S = sum ln x.  ln x >= ln 2 > 1/2 for x >= 2, so every
// FP64 ln x is an integer multiple of 2^-53 and ln x * 2^53 is an exact
// integer below 2^59.  Summing those integers in 128 bits is exact in any
// order, which makes S independent of how draws are split across lanes.
// ---------------------------------------------------------------------------
struct U128 {
  uint64_t lo, hi;
};

ZPL_HD void u128_add(U128& a, uint64_t lo, uint64_t hi) {
  const uint64_t s = a.lo + lo;
  a.hi += hi + (s < lo ? 1u : 0u);
  a.lo = s;
}

// c * L (c < 2^32, L < 2^60) added exactly.
ZPL_HD void u128_add_mul(U128& a, uint64_t c, uint64_t L) {
  const uint64_t ll = (L & 0xffffffffull) * c;
  const uint64_t lh = (L >> 32) * c;  // < 2^60
  // c*L = lh * 2^32 + ll
  u128_add(a, ll, 0);
  u128_add(a, lh << 32, lh >> 32);
}

ZPL_HD uint64_t ln_fixed(int64_t v, const double* __restrict__ ln) {
  return v <= 1 ? 0ull : (uint64_t)(ln_value(v, ln) * 0x1p53);
}

// Deterministic FP64 value of a 128-bit fixed-point sum (unit 2^-53).
ZPL_HD double u128_to_S(const U128& a) {
  double v = (a.hi == 0) ? (double)a.lo : fma((double)a.hi, 0x1p64, (double)a.lo);
  return v * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Double-double arithmetic (Dekker; Bailey's QD formulation) for the exact
// integer floor in the tail sampler.
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};

ZPL_HD DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return DD{s, e};
}
ZPL_HD DD quick_two_sum(double a, double b) {
  const double s = a + b;
  return DD{s, b - (s - a)};
}
ZPL_HD DD two_prod(double a, double b) {
  const double p = a * b;
  return DD{p, fma(a, b, -p)};
}
ZPL_HD DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  DD t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
// a + b when they do not cancel (|a + b| not far below max(|a|, |b|)):
// absolute error about 2^-105 max(|a|, |b|).
ZPL_HD DD dd_add_nc(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return quick_two_sum(s.hi, s.lo);
}
ZPL_HD DD dd_mul(DD a, DD b) {
  DD p = two_prod(a.hi, b.hi);
  p.lo = fma(a.hi, b.lo, p.lo);
  p.lo = fma(a.lo, b.hi, p.lo);
  return quick_two_sum(p.hi, p.lo);
}
ZPL_HD DD dd_mul_d(DD a, double b) {
  DD p = two_prod(a.hi, b);
  p.lo = fma(a.lo, b, p.lo);
  return quick_two_sum(p.hi, p.lo);
}
ZPL_HD DD dd_div_d(DD a, double b) {
  const double q1 = a.hi / b;
  DD r = dd_add(a, dd_mul_d(DD{q1, 0.0}, -b));
  const double q2 = r.hi / b;
  r = dd_add(r, dd_mul_d(DD{q2, 0.0}, -b));
  const double q3 = r.hi / b;
  DD q = quick_two_sum(q1, q2);
  return dd_add(q, DD{q3, 0.0});
}

// exp of a double-double (|a| < 900): a = (64 q + j) ln2/64 + r with
// 0 <= j < 64 and |r| <= ln2/128 (ln2/64 in three parts, the first short
// enough for k ln2/64 to be exact), exp(a) = 2^q 2^(j/64) exp(r) with
// 2^(j/64) from a double-double table.  exp(r) - 1 by Horner: the terms from
// r^6/6! on (below 2^-54 of the sum) in FP64, the rest in double-double.
// Every addition is between terms that do not cancel (the reduction's
// correction k L2 is below 2^-28 and far from the result unless r itself is
// that small, where only its absolute error counts).  Relative error about
// 2^-104.
ZPL_HD DD dd_exp(DD a) {
  const double k = rint(a.hi * kInvLn2by64);
  // a.hi - k L1 is exact: k L1 has at most 53 bits and lies within |r| of a.hi
  DD r = two_sum(fma(-k, kLn2by64[0], a.hi), a.lo);
  r = dd_add_nc(r, two_prod(-k, kLn2by64[1]));
  r = quick_two_sum(r.hi, r.lo - k * kLn2by64[2]);
  const double x = r.hi;
  const double u =
      1.0 / 720.0 +
      x * (1.0 / 5040.0 +
           x * (1.0 / 40320.0 + x * (1.0 / 362880.0 + x * (1.0 / 3628800.0 + x / 39916800.0))));
  DD p = dd_add_nc(DD{kInvFact5Hi, kInvFact5Lo}, dd_mul_d(r, u));
  p = dd_add_nc(DD{kInvFact4Hi, kInvFact4Lo}, dd_mul(r, p));
  p = dd_add_nc(DD{kInvFact3Hi, kInvFact3Lo}, dd_mul(r, p));
  p = dd_add_nc(DD{0.5, 0.0}, dd_mul(r, p));
  const DD em1 = dd_add_nc(r, dd_mul(dd_mul(r, r), p));  // exp(r) - 1
  const int ki = (int)k;
  const int j = ki & 63;
  const int q = (ki - j) / 64;
  const DD t = {kExp2Hi[j], kExp2Lo[j]};
  const DD e = dd_add_nc(t, dd_mul(t, em1));
  return DD{ldexp(e.hi, q), ldexp(e.lo, q)};
}

// ln of a positive double as a double-double: one Newton step on exp from
// y = log(v), ln v = y + ln(1 + t) with t = v exp(-y) - 1 (|t| about the
// error of y, so t - t^2/2 suffices; the square matters when |y| is large).
// v exp(-y) is within 2^-40 of 1, so subtracting 1 from its high part is
// exact.
ZPL_HD DD dd_log(double v) {
  const double y = log(v);
  const DD p = dd_mul_d(dd_exp(DD{-y, 0.0}), v);
  const DD t = two_sum(p.hi - 1.0, p.lo);
  return dd_add_nc(DD{y, 0.0}, quick_two_sum(t.hi, t.lo - 0.5 * t.hi * t.hi));
}

// ---------------------------------------------------------------------------
// Guide table over the uniform (layout in zpl_kernels.hpp).  The sampler
// compares the uniform's odd 53-bit integer m (U = m 2^-53) with the table as
// integers TI[k] = floor(T[k] 2^53): F(k) >= U exactly when TI[k] >= m.
// ---------------------------------------------------------------------------
ZPL_HD uint64_t table_int(double t) { return (uint64_t)(t * 0x1p53); }

// Guide bin of U = m 2^-53 with sh refinement bits.  U < 1/2: kGA bins
// uniform in U, bin m >> 44.  U > 1/2: e = 1 - U = (2^53 - m) 2^-53 exactly;
// the bin is given by the octave and the top kGBits + sh mantissa bits of e,
// which are the biased exponent and mantissa fields of the double (2^53 - m)
// (exact, < 2^53) shifted by 53 octaves; bins past the last entry (octaves
// of e below the table's end: tail draws, when sh > 0) are clamped to it.
// Both parts are computed and one selected.
ZPL_HD int guide_index(uint64_t m, int sh) {
  const bool uni = sh == kGuideUniform;  // the uniform layout: bin m >> 42 for every m
  const uint32_t mh = (uint32_t)(m >> 32);
  const int ia = (int)(mh >> (uni ? 10 : 12));
  const uint32_t lim = uni ? (1u << 21) : (1u << 20);
  // e = 2^53 - m as a double, exactly: (2^53 - low word) - high word 2^32
  const double e = fma(-(double)mh, 0x1p32, 0x1p53 - (double)(uint32_t)m);
  const int nb = kGBits + (uni ? 0 : sh);
  const int q = (int)((uint32_t)(__builtin_bit_cast(uint64_t, e) >> 32) >> (20 - nb));
  // bin = kGA + ((1021 - E) << nb) + (2^nb - 1 - s) for e = 2^(E-1023)(1.s...),
  // and q = ((E + 53) << nb) | s
  const int ib = kGA + ((1074 << nb) + ((1 << nb) - 1)) - q;
  const int ibc = ib < kGuide - 1 ? ib : kGuide - 1;
  return mh < lim ? ia : ibc;
}

// The refinement of a cell's log-scale guide: the largest sh <= kGuideShMax
// whose 52 >> sh octaves of e still reach the octave of the table's end
// (e = 2^53 - timax, rounded to the next odd m: conservative), so that every
// uniform that is not a tail draw has an unclamped bin.
ZPL_HD int guide_refinement(uint64_t timax) {
  if (timax < (1ull << 52)) return 0;
  const uint64_t mt = (timax < (1ull << 53) - 1 ? timax : (1ull << 53) - 1) | 1ull;
  const int o_last = (guide_index(mt, 0) - kGA) >> kGBits;
  int sh = 0;
  for (int s = 1; s <= kGuideShMax; ++s)
    if (((o_last + 1) << (kGBits + s)) <= kGuide - kGA) sh = s;
  return sh;
}

// First index k in T[0..kH) with T[k] >= t (kH when none).
ZPL_HD int table_lower_bound(const double* T, double t) {
  int lo = 0, hi = kH;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (T[mid] >= t)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// The cell's guide layout: the uniform one for a bounded support (no tail,
// T[kH] = 1) whose values between the median and the upper quartile span
// more than the 64 log-scale bins of that octave of U (the truncated law at
// small exponents, nearly uniform on 1..K, where the log bins are several
// values wide); else the log-scale layout with guide_refinement.
ZPL_HD int guide_layout(const double* T) {
  const uint64_t timax = table_int(T[kH - 1]);
  if (timax >= (1ull << 53) &&
      table_lower_bound(T, 0.75) - table_lower_bound(T, 0.5) > (1 << kGBits))
    return kGuideUniform;
  return guide_refinement(timax);
}

// The smallest m a uniform in bin b (0 <= b < kGuide) can have, in integers
// (a bin of the U > 1/2 part can be narrower than the spacing of doubles
// near 1, where 1 - e rounds).  In units of 2^-53 the bin's e lies below
// e_hi = (2^nb + s + 1) 2^(51 - o - nb), so its largest integer e is
// (2^nb + s) >> (o + nb - 51), or e_hi - 1 when e_hi is an integer.  The
// guide entry is then 1 + the first index k with TI[k] >= guide_bin_min(b).
ZPL_HD uint64_t guide_bin_min(int b, int sh) {
  if (sh == kGuideUniform) return b < 2048 ? (uint64_t)b << 42 : (1ull << 53);
  if (b < kGA) return (uint64_t)b << 44;
  const int nb = kGBits + sh;
  const int o = (b - kGA) >> nb;
  const int s = ((1 << nb) - 1) - ((b - kGA) & ((1 << nb) - 1));
  const uint64_t N = (1ull << nb) + (uint64_t)s + 1ull;
  const int k = o + nb - 51;
  const uint64_t emax = k >= 0 ? ((N - 1ull) >> k) : ((N << (-k)) - 1ull);
  return (1ull << 53) - emax;
}

// Packed guide entry of bin b for the simulation's fast path, from the guide
// g[0..kGuide] (brackets [g[b], g[b + 1]]): the bracket low lo in bits 0..15;
// bits 16..31 hold the bracket high hi when the bracket is exactly two wide
// and the bin holds no tail uniform, else kDeferred | hi.  Bin b holds the m
// in [guide_bin_min(b), guide_bin_min(b + 1)) (the last bin: up to 2^53), so
// it may hold a tail uniform (m > timax) when that range reaches above timax.
constexpr int kDeferred = 0x8000;
static_assert(kH + 1 < kDeferred, "bracket bounds fit below the deferral mark");

ZPL_HD uint32_t guide_pack(const uint16_t* g, int b, int sh, uint64_t timax) {
  const uint32_t lo = g[b], hi = g[b + 1];
  const uint64_t mend = b + 1 < kGuide ? guide_bin_min(b + 1, sh) : (1ull << 53);
  const bool tail = mend - 1 > timax;
  const uint32_t hw = (hi == lo + 1 && !tail) ? hi : ((uint32_t)kDeferred | hi);
  return lo | (hw << 16);
}

// ---------------------------------------------------------------------------
// Tail sampler for U > T[kH].  Target on k >= m = kH + 1: p(k) ~ k^-a.
// Proposal X = floor(Y), Y = m V^(-1/beta) (Pareto, beta = a - 1), so
// P(X = k) ~ k^-beta - (k+1)^-beta; the ratio target/proposal is proportional
// to g(k) = 1 / (k (1 - (1+1/k)^-beta)), decreasing in k, so X is accepted
// when W g(m) <= g(X).  Y >= 2^63 is redrawn (law conditioned on x < 2^63).
// X is the exact floor of the real-number Y: FP64 decides it unless Y is
// within a relative 2^-44 of an integer (or of 2^63) or above 2^52, where
// the floor is taken from a double-double evaluation of Y.
// ---------------------------------------------------------------------------
ZPL_HD double tail_g(double beta, double k) {
  return 1.0 / (-k * expm1(-beta * log1p(1.0 / k)));
}

ZPL_HD int64_t dd_floor(DD y) {
  const double f = floor(y.hi);
  // callers guarantee y < 2^63; y.hi may still round up to 2^63
  if (f >= 0x1p63) return (int64_t)0x7fffffffffffffffll;
  if (f == y.hi) {
    // y.hi is an integer (always so above 2^52): floor(y) = y.hi + floor(y.lo),
    // |y.lo| <= ulp(y.hi)/2 <= 2^9
    return (int64_t)f + (int64_t)floor(y.lo);
  }
  // y.hi < 2^52 is not an integer and |y.lo| < 1/2
  int64_t X = (int64_t)f;
  const double frac = (y.hi - f) + y.lo;
  if (frac < 0.0) X -= 1;
  if (frac >= 1.0) X += 1;
  return X;
}

// The floor of Y = m0 V^(-1/beta) from a double-double evaluation, for the
// proposals FP64 cannot decide (above 2^52 or within a relative 2^-44 of an
// integer or of 2^63): false when Y >= 2^63 (the proposal is redrawn).  Out
// of line: rare, and long (two double-double exponentials).
static __host__ __device__ __noinline__ bool tail_floor_dd(double V, double beta, double m0,
                                                           int64_t* X) {
  const DD zd = dd_div_d(dd_log(V), -beta);
  const DD Y = dd_mul_d(dd_exp(zd), m0);
  if (Y.hi > 0x1p63 || (Y.hi == 0x1p63 && Y.lo >= 0.0)) return false;
  *X = dd_floor(Y);
  return true;
}

// Returns the accepted draw; ORs kFlagTailCapped into *flags if a proposal at
// or above 2^63 was rejected.
// Rejection tail on k >= m0 (m0 an integer below 2^53): kTailM for the pure
// law, xmin + kH for the law with a lower cutoff; gm = tail_g(beta, m0).
ZPL_HD int64_t tail_draw_from(double m0, double beta, double gm, uint32_t k0, uint32_t k1,
                              uint32_t i, uint32_t rep, uint32_t stream, uint32_t* flags) {
  const double two63 = 0x1p63;
  for (uint32_t attempt = 0; attempt < 0x7fffffffu; ++attempt) {
    const Words4 w = philox4x32_10(i, rep, stream, kTailDomain | attempt, k0, k1);
    const double V = u53(w.w0, w.w1);
    const double W = u53(w.w2, w.w3);
    const double z = -log(V) / beta;
    const double y = m0 * exp(z);
    int64_t X;
    if (y >= two63 * (1.0 + 0x1p-40)) {
      *flags |= kFlagTailCapped;
      continue;
    }
    const double fy = floor(y);
    const double tol = y * 0x1p-44;
    if (y < 0x1p52 && y < two63 * (1.0 - 0x1p-40) && (y - fy) > tol &&
        (fy + 1.0 - y) > tol) {
      X = (int64_t)fy;
    } else if (!tail_floor_dd(V, beta, m0, &X)) {
      *flags |= kFlagTailCapped;
      continue;
    }
    // g(k) >= 1/beta for every k ((1 + t)^-beta >= 1 - beta t), and the FP64
    // tail_g is within a few ulps of the truth: a proposal with
    // W g(m0) beta <= 1 - 2^-39 passes the full test too, which is skipped
    // (about 99.98 % of proposals; the decision is the same either way)
    const double wg = W * gm;
    if (wg * beta <= 1.0 - 0x1p-39 || wg <= tail_g(beta, (double)X)) return X;
  }
  return (int64_t)m0;
}

ZPL_HD int64_t tail_draw(double beta, double gm, uint32_t k0, uint32_t k1,
                         uint32_t i, uint32_t rep, uint32_t stream, uint32_t* flags) {
  return tail_draw_from(kTailM, beta, gm, k0, k1, i, rep, stream, flags);
}

}  // namespace zpl
