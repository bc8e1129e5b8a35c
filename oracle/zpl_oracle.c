/*
 * zpl_oracle.c -- reference (oracle) implementation, TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of what the GPU library
 * computes, written from Rappos & Robert, "Using GPU Simulation to Accurately
 * Fit to the Power-Law Distribution" (2013).  It exists to check the GPU path
 * against; nothing in the product may call it.  Every floating-point step is
 * FP64 (the paper insists on double precision in Sect. 4), except one integer
 * floor in the rejection tail, taken in quad precision so that the integer it
 * produces is the exact floor of the real-number formula.
 *
 * Per replicate (Sect. 3 and Sect. 4 of the paper):
 *   1. draw n integers from p(k) = k^-alpha / zeta(alpha), k >= 1   (eq. 1)
 *   2. solve zeta'(a)/zeta(a) = -(1/n) sum ln x_i for a = alpha_hat (eq. 2)
 *   3. D = sup_x |F(x; alpha_hat) - S_n(x)|                        (eq. 3)
 * and the replicates of a cell are reduced to order statistics of D.
 *
 * Conventions that the paper leaves open (each is a documented reading):
 *   - RNG: Philox4x32-10, key = (seed lo, seed hi), counter =
 *     (draw block j, replicate, stream, domain).  Domain 0: body draws, block
 *     j gives draws 2j (words 0,1) and 2j+1 (words 2,3).  Domain
 *     0x80000000|attempt with counter word 0 = draw index: tail proposals.
 *   - U = ((w_hi:w_lo >> 11) | 1) * 2^-53, an odd multiple of 2^-53 in (0,1).
 *   - Body: x = min{k in 1..H : T[k] >= U}, T[k] = F(k; alpha), H = 4096;
 *     the ">=" tie rule is the annex sampler's.
 *   - Tail (U > T[H]): rejection from the floored Pareto envelope on k >= H+1,
 *     conditioned on x < 2^63 (proposals at or above 2^63 are redrawn).
 *   - All-ones rule: if every draw is 1 (S = 0), S is replaced by ln 2, the
 *     annex's adjustment (one of the points is counted as a 2).
 *   - MLE solved to full FP64 precision (the annex stops at 1e-5).
 *   - KS sup taken over all integers t >= 0 (equivalently all real x).
 *   - Quantile: ascending order statistic at 0-based index floor(R*num/den),
 *     the annex's integer index rule.
 *   - Bootstrap p-value: #{D_b >= D_obs} / B.
 */
#define _GNU_SOURCE
#include "zpl_oracle.h"

#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel     */
/* random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of the S-box      */
/* (two 32x32->64 multiplies, xor with the key) with a Weyl key schedule.    */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

double orc_u53(uint32_t hi, uint32_t lo) {
  uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
  uint64_t m = (w >> 11) | 1u;
  return (double)m * 0x1p-53;
}

/* ------------------------------------------------------------------------ */
/* Zeta functions.  The paper gives zeta only as the infinite sum (Sect. 1). */
/* It is evaluated here by the Euler-Maclaurin formula for the Hurwitz zeta  */
/*   zeta(s,q) = sum_{j<N} (q+j)^-s + a^(1-s)/(s-1) + a^-s/2                 */
/*             + sum_{i=1..P} B_2i/(2i)! * s(s+1)..(s+2i-2) * a^(-s-2i+1),   */
/* a = q + N, and its term-by-term s-derivatives.                            */
/* ------------------------------------------------------------------------ */
#define ORC_EM_N 20
#define ORC_EM_P 10

/* Bernoulli numbers B_2 .. B_20 as exact rationals. */
static const double bern_num[ORC_EM_P] = {1.0,     -1.0,   1.0,     -1.0,
                                          5.0,     -691.0, 7.0,     -3617.0,
                                          43867.0, -174611.0};
static const double bern_den[ORC_EM_P] = {6.0,  30.0,   42.0, 30.0,  66.0,
                                          2730.0, 6.0, 510.0, 798.0, 330.0};

static double em_coef(int i /* 1-based */) {
  double fact = 1.0; /* (2i)! */
  for (int k = 2; k <= 2 * i; ++k) fact *= (double)k;
  return bern_num[i - 1] / (bern_den[i - 1] * fact);
}

/* zeta(s, q) and its first two s-derivatives, each multiplied by r^s (r > 0):
 * every power x^-s is taken as (x/r)^-s = exp(-s log1p((x - r)/r)), while the
 * logarithms ln x the derivatives bring down stay as they are.  The factor r^s
 * is common to all three and cancels in every ratio the method uses (the
 * likelihood equation (2) and the CDF of eq. (1)); with r = xmin it keeps the
 * sums representable, where x^-s alone underflows for s ln x > 708.  r = 1
 * gives the plain values. */
static double pow_rel(double x, double r, double s) {
  return r == 1.0 ? pow(x, -s) : exp(-s * log1p((x - r) / r));
}

void orc_hurwitz3_scaled(double s, double q, double r, double out[3]) {
  const double a = q + (double)ORC_EM_N;
  const double L = log(a);
  const double sm1 = s - 1.0;
  const double as = pow_rel(a, r, s);                             /* (a/r)^(-s)  */
  const double a1s = r == 1.0 ? pow(a, 1.0 - s) : a * as;         /* a^(1-s) r^s */
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;

  /* Bernoulli correction terms, smallest first. */
  double tb0[ORC_EM_P], tb1[ORC_EM_P], tb2[ORC_EM_P];
  {
    double P = s;             /* s (s+1) ... (s+m-1), m = 2i-1 */
    double sig1 = 1.0 / s;    /* sum 1/(s+k)   */
    double sig2 = 1.0 / (s * s); /* sum 1/(s+k)^2 */
    double E = as / a;        /* a^(-s-m) */
    int m = 1;
    for (int i = 1; i <= ORC_EM_P; ++i) {
      double c = em_coef(i);
      double P1 = P * sig1;
      double P2 = P * (sig1 * sig1 - sig2);
      tb0[i - 1] = c * P * E;
      tb1[i - 1] = c * (P1 - L * P) * E;
      tb2[i - 1] = c * (P2 - 2.0 * L * P1 + L * L * P) * E;
      /* advance m -> m + 2 */
      double u = s + (double)m, v = s + (double)(m + 1);
      P *= u * v;
      sig1 += 1.0 / u + 1.0 / v;
      sig2 += 1.0 / (u * u) + 1.0 / (v * v);
      E /= a * a;
      m += 2;
    }
  }
  for (int i = ORC_EM_P - 1; i >= 0; --i) {
    z0 += tb0[i];
    z1 += tb1[i];
    z2 += tb2[i];
  }
  /* a^-s / 2 */
  z0 += 0.5 * as;
  z1 += -0.5 * L * as;
  z2 += 0.5 * L * L * as;
  /* integral a^(1-s)/(s-1) */
  z0 += a1s / sm1;
  z1 += a1s * (-L / sm1 - 1.0 / (sm1 * sm1));
  z2 += a1s * (L * L / sm1 + 2.0 * L / (sm1 * sm1) + 2.0 / (sm1 * sm1 * sm1));
  /* direct terms, largest index (smallest term) first */
  for (int j = ORC_EM_N - 1; j >= 0; --j) {
    double x = q + (double)j;
    double lx = log(x);
    double t = pow_rel(x, r, s);
    z0 += t;
    z1 += -lx * t;
    z2 += lx * lx * t;
  }
  out[0] = z0;
  out[1] = z1;
  out[2] = z2;
}

void orc_hurwitz3(double s, double q, double out[3]) { orc_hurwitz3_scaled(s, q, 1.0, out); }

void orc_zeta3(double s, double out[3]) { orc_hurwitz3(s, 1.0, out); }

static double hurwitz0(double s, double q) {
  double z[3];
  orc_hurwitz3(s, q, z);
  return z[0];
}

/* zeta(s, q) r^s (see orc_hurwitz3_scaled). */
static double hurwitz0_rel(double s, double q, double r) {
  double z[3];
  orc_hurwitz3_scaled(s, q, r, z);
  return z[0];
}

/* F(t; alpha) = sum_{k<=t} k^-alpha / zeta(alpha) = 1 - zeta(alpha,t+1)/zeta(alpha). */
double orc_cdf(double alpha, int64_t t) {
  if (t <= 0) return 0.0;
  return 1.0 - hurwitz0(alpha, (double)t + 1.0) / hurwitz0(alpha, 1.0);
}

void orc_cdf_table(double alpha, double *T, int H) {
  double z = hurwitz0(alpha, 1.0);
  for (int k = 1; k <= H; ++k)
    T[k - 1] = 1.0 - hurwitz0(alpha, (double)k + 1.0) / z;
}

/* ------------------------------------------------------------------------ */
/* Sampling (eq. 1).  Body: inverse CDF against T with the ">=" tie rule.    */
/* Tail: the law restricted to k >= m = H+1 has p(k) proportional to         */
/* k^-alpha.  Proposal X = floor(Y), Y Pareto on [m, inf) with index          */
/* beta = alpha-1, i.e. Y = m V^(-1/beta); P(X = k) is proportional to        */
/* k^-beta - (k+1)^-beta.  The ratio target/proposal is proportional to       */
/* g(k) = 1 / (k (1 - (1+1/k)^-beta)), which decreases in k, so X is          */
/* accepted with probability g(X)/g(m), i.e. when W g(m) <= g(X).  Proposals  */
/* with Y >= 2^63 are rejected, which conditions the law on x < 2^63.         */
/* ------------------------------------------------------------------------ */
static double tail_g(double beta, double k) {
  return 1.0 / (-k * expm1(-beta * log1p(1.0 / k)));
}

int64_t orc_tail_draw(double alpha, uint64_t seed, uint32_t stream,
                         uint32_t rep, uint32_t i, uint32_t *flags) {
  const double beta = alpha - 1.0; /* exact in FP64 for alpha > 1 */
  const double m = (double)(ORC_TABLE_H + 1);
  const double gm = tail_g(beta, m);
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const __float128 two63 = 9223372036854775808.0Q;
  for (uint32_t attempt = 0; attempt < 0x7fffffffu; ++attempt) {
    uint32_t ctr[4] = {i, rep, stream, 0x80000000u | attempt};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double V = orc_u53(w[0], w[1]);
    double W = orc_u53(w[2], w[3]);
    __float128 Y = (__float128)m * expq(-logq((__float128)V) / (__float128)beta);
    if (Y >= two63) {
      *flags |= ORC_FLAG_TAIL_CAPPED;
      continue;
    }
    int64_t X = (int64_t)floorq(Y);
    if (W * gm <= tail_g(beta, (double)X)) return X;
  }
  return ORC_TABLE_H + 1; /* unreachable in practice */
}

int64_t orc_draw(double alpha, const double *T, uint64_t seed, uint32_t stream,
                 uint32_t rep, uint32_t i, uint32_t *flags) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {i >> 1, rep, stream, 0u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double U = (i & 1u) ? orc_u53(w[2], w[3]) : orc_u53(w[0], w[1]);
  if (U > T[ORC_TABLE_H - 1]) return orc_tail_draw(alpha, seed, stream, rep, i, flags);
  /* smallest k with T[k] >= U (binary search over the nondecreasing table) */
  int lo = 1, hi = ORC_TABLE_H;
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (T[mid - 1] >= U)
      hi = mid;
    else
      lo = mid + 1;
  }
  return (int64_t)lo;
}

void orc_sample(double alpha, const double *T, int64_t n, uint64_t seed,
                uint32_t stream, uint32_t rep, int64_t *x, uint32_t *flags) {
  for (int64_t i = 0; i < n; ++i)
    x[i] = orc_draw(alpha, T, seed, stream, rep, (uint32_t)i, flags);
}

/* ------------------------------------------------------------------------ */
/* MLE (Sect. 2, eq. 2): solve g(a) = -zeta'(a)/zeta(a) - m = 0.  g is       */
/* strictly decreasing (g' = -Var[ln X] under the law with exponent a), so   */
/* the root is unique.  Newton-Raphson as the paper prescribes, kept inside   */
/* a bracket [1 + 2^-20, 64] that shrinks with the sign of g; a step leaving  */
/* the bracket is replaced by bisection.                                     */
/* ------------------------------------------------------------------------ */
/* Reading shared by the three laws (pure, truncated, with a cutoff): eq. 2   */
/* is solved to FP64 precision.  The iteration stops after a step of at most */
/* 2^-40 max(|a|, 1) and returns the next iterate (Newton converges          */
/* quadratically, so that iterate sits at the rounding noise of mu); after   */
/* ORC_MLE_CAP iterations it stops, and NOCONV is set only when the last     */
/* residual |mu(a) - m| exceeds 2^-44 m, the rounding noise of an FP64 mu:   */
/* NOCONV means that no root was found, never rounding noise.                */
#define ORC_MLE_CAP 200
static _Thread_local int orc_iters;
int orc_mle_last_iters(void) { return orc_iters; }

double orc_mle(double m, uint32_t *flags) {
  orc_iters = 0;
  double lo = 1.0 + 0x1p-20, hi = 64.0;
  double a = 1.0 + 1.0 / m; /* from -zeta'/zeta ~ 1/(a-1) near a = 1 */
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  double g_last = 0.0;
  for (int it = 0; it < ORC_MLE_CAP; ++it) {
    orc_iters = it + 1;
    double z[3];
    orc_zeta3(a, z);
    double r1 = z[1] / z[0];
    double g = -r1 - m;
    if (g == 0.0) return a;
    g_last = g;
    if (g > 0.0)
      lo = a;
    else
      hi = a;
    double gp = -(z[2] / z[0] - r1 * r1);
    double an = a - g / gp;
    /* closed bracket: a converged Newton step may land exactly on lo or hi */
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= ORC_FLAG_BISECT;
    }
    if (fabs(an - a) <= 0x1p-40 * a) return an;
    a = an;
  }
  if (!(fabs(g_last) <= 0x1p-44 * m)) *flags |= ORC_FLAG_NOCONV;
  return a;
}

/* ------------------------------------------------------------------------ */
/* Fit one dataset: S, alpha_hat and the KS distance (eq. 3).                */
/* Both CDFs are right-continuous step functions jumping only at integers,   */
/* so the sup over real x is a max over integers t >= 0.  Between two         */
/* consecutive distinct sample values v' < v, S_n is constant and F rises,   */
/* so |F - S_n| peaks at t = v' or t = v - 1; beyond the largest value,       */
/* |1 - F| decreases.  Hence D = max over distinct v of                       */
/*   |C(v)/n - F(v)| and |C(v-1)/n - F(v-1)|,  C = count of draws <= t.       */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static double neumaier_sum_log(const int64_t *xs, int64_t n) {
  double sum = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = log((double)xs[i]);
    double t = sum + v;
    if (fabs(sum) >= fabs(v))
      c += (sum - t) + v;
    else
      c += (v - t) + sum;
    sum = t;
  }
  return sum + c;
}

static double ks_sorted(const int64_t *xs, int64_t n, double a) {
  const double z = hurwitz0(a, 1.0);
  const double dn = (double)n;
  double D = 0.0;
  int64_t i = 0;
  while (i < n) {
    int64_t v = xs[i];
    int64_t below = i; /* draws < v, i.e. C(v-1) */
    while (i < n && xs[i] == v) ++i;
    int64_t upto = i; /* C(v) */
    double Fv = 1.0 - hurwitz0(a, (double)v + 1.0) / z;
    double Fv1 = (v - 1 <= 0) ? 0.0 : 1.0 - hurwitz0(a, (double)v) / z;
    double d1 = fabs((double)upto / dn - Fv);
    double d2 = fabs((double)below / dn - Fv1);
    if (d1 > D) D = d1;
    if (d2 > D) D = d2;
  }
  return D;
}

/* xs must be sorted ascending; fills S (after the all-ones rule), a, D. */
static void fit_sorted(const int64_t *xs, int64_t n, double *S, double *ahat,
                       double *D, uint32_t *flags) {
  double s = neumaier_sum_log(xs, n);
  if (s == 0.0) { /* all draws are 1 */
    s = log(2.0);
    *flags |= ORC_FLAG_ALL_ONES;
  }
  double a = orc_mle(s / (double)n, flags);
  *S = s;
  *ahat = a;
  *D = ks_sorted(xs, n, a);
}

int orc_fit(const int64_t *x, int64_t n, double *S, double *alpha_hat,
            double *D, uint32_t *flags) {
  if (n < 1) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (x[i] < 1) return -1;
  int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!xs) return -1;
  memcpy(xs, x, sizeof(int64_t) * (size_t)n);
  qsort(xs, (size_t)n, sizeof(int64_t), cmp_i64);
  uint32_t f = 0;
  fit_sorted(xs, n, S, alpha_hat, D, &f);
  *flags = f;
  free(xs);
  return 0;
}

/* splitmix64's output finaliser (Steele, Lea and Flood, OOPSLA 2014). */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Replicates of one cell, split statically over threads.                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  double alpha;
  int64_t n;
  uint64_t seed;
  uint32_t stream;
  int64_t rep_lo, count;
  const double *T;
  double *D, *ahat, *S;
  uint32_t *flags;
  uint64_t *fp;
  int64_t *xmax;
  int64_t begin, end; /* slice of [0, count) */
} sim_job;

static void *sim_worker(void *arg) {
  sim_job *j = (sim_job *)arg;
  int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)(j->n > 0 ? j->n : 1));
  for (int64_t r = j->begin; r < j->end; ++r) {
    uint32_t rep = (uint32_t)(j->rep_lo + r);
    uint32_t f = 0;
    orc_sample(j->alpha, j->T, j->n, j->seed, j->stream, rep, x, &f);
    uint64_t h = 0;
    for (int64_t i = 0; i < j->n; ++i) h += mix64((uint64_t)x[i]);
    qsort(x, (size_t)j->n, sizeof(int64_t), cmp_i64);
    double s, a, d;
    fit_sorted(x, j->n, &s, &a, &d, &f);
    if (j->D) j->D[r] = d;
    if (j->ahat) j->ahat[r] = a;
    if (j->S) j->S[r] = s;
    if (j->flags) j->flags[r] = f;
    if (j->fp) j->fp[r] = h;
    if (j->xmax) j->xmax[r] = x[j->n - 1];
  }
  free(x);
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

int orc_simulate(double alpha, int64_t n, uint64_t seed, uint32_t stream,
                 int64_t rep_lo, int64_t count, double *D, double *alpha_hat,
                 double *S, uint32_t *flags, uint64_t *fp, int64_t *xmax,
                 int nthreads) {
  if (n < 1 || count < 0 || !(alpha > 1.0)) return -1;
  double *T = (double *)malloc(sizeof(double) * ORC_TABLE_H);
  if (!T) return -1;
  orc_cdf_table(alpha, T, ORC_TABLE_H);
  int nt = resolve_threads(nthreads);
  if (nt > count) nt = count > 0 ? (int)count : 1;
  sim_job *jobs = (sim_job *)calloc((size_t)nt, sizeof(sim_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; ++t) {
    sim_job *j = &jobs[t];
    j->alpha = alpha;
    j->n = n;
    j->seed = seed;
    j->stream = stream;
    j->rep_lo = rep_lo;
    j->count = count;
    j->T = T;
    j->D = D;
    j->ahat = alpha_hat;
    j->S = S;
    j->flags = flags;
    j->fp = fp;
    j->xmax = xmax;
    j->begin = count * t / nt;
    j->end = count * (t + 1) / nt;
    if (nt == 1)
      sim_worker(j);
    else
      pthread_create(&th[t], NULL, sim_worker, j);
  }
  if (nt > 1)
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free(T);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Quantiles: the annex sorts the D values and reads index R*q with integer  */
/* arithmetic (R*9/10, R*95/100, ...).                                       */
/* ------------------------------------------------------------------------ */
static int cmp_f64(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

double orc_quantile(const double *D, int64_t R, uint32_t num, uint32_t den) {
  if (R < 1 || den == 0 || num >= den) return NAN;
  double *s = (double *)malloc(sizeof(double) * (size_t)R);
  memcpy(s, D, sizeof(double) * (size_t)R);
  qsort(s, (size_t)R, sizeof(double), cmp_f64);
  uint64_t idx = ((uint64_t)R * (uint64_t)num) / (uint64_t)den;
  double v = s[idx];
  free(s);
  return v;
}

/* ------------------------------------------------------------------------ */
/* Bespoke cutoff (Sect. 4): simulate at the sample's own (n, alpha_hat),    */
/* refitting every replicate by MLE, and report the fraction of replicates   */
/* whose D is at least the observed one.                                     */
/* ------------------------------------------------------------------------ */
int orc_bootstrap_pvalue(const int64_t *x, int64_t n, int64_t B, uint64_t seed,
                         uint32_t stream, double *alpha_hat, double *D,
                         double *p, uint32_t *flags, int nthreads) {
  if (B < 1) return -1;
  double S, a, d;
  uint32_t f = 0;
  if (orc_fit(x, n, &S, &a, &d, &f) != 0) return -1;
  double *Db = (double *)malloc(sizeof(double) * (size_t)B);
  if (!Db) return -1;
  if (orc_simulate(a, n, seed, stream, 0, B, Db, NULL, NULL, NULL, NULL, NULL,
                   nthreads) != 0) {
    free(Db);
    return -1;
  }
  int64_t ge = 0;
  for (int64_t b = 0; b < B; ++b)
    if (Db[b] >= d) ++ge;
  free(Db);
  *alpha_hat = a;
  *D = d;
  *p = (double)ge / (double)B;
  *flags = f;
  return 0;
}

/* ======================================================================== */
/* The truncated law (Sect. 1 with a finite upper limit K; Tables 2-6):      */
/* p(k) = k^-g / Z_K(g) for k = 1..K, Z_K(g) = sum_{k=1..K} k^-g.  Every sum */
/* is taken directly from its definition (largest index first).  The law is  */
/* defined for every real g; the tables use g > 0, and the MLE may fall at   */
/* or below 0 for a sample with many large values.                           */
/* ======================================================================== */

/* suf[t] = sum_{k=t+1..K} k^-g for t = 0..K, so suf[0] = Z_K(g), suf[K] = 0. */
static void tz_suffix(double g, int K, double *suf) {
  suf[K] = 0.0;
  for (int t = K - 1; t >= 0; --t) suf[t] = suf[t + 1] + pow((double)(t + 1), -g);
}

void orc_tz_norm3(double g, int K, double out[3]) {
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  for (int k = K; k >= 1; --k) {
    const double t = pow((double)k, -g), l = log((double)k);
    z0 += t;
    z1 -= l * t;
    z2 += l * l * t;
  }
  out[0] = z0;
  out[1] = z1;
  out[2] = z2;
}

int orc_tz_cdf_table(double g, int K, double *T) {
  if (K < 2) return -1;
  double *suf = (double *)malloc(sizeof(double) * (size_t)(K + 1));
  if (!suf) return -1;
  tz_suffix(g, K, suf);
  for (int k = 1; k <= K; ++k) T[k - 1] = 1.0 - suf[k] / suf[0];
  free(suf);
  return 0;
}

/* Draw i of replicate `rep`: the counter layout of the pure law's body     */
/* draws; x = min{k in 1..K : T[k] >= U}.  T[K] = 1 > U, so there is no tail. */
int64_t orc_tz_draw(const double *T, int K, uint64_t seed, uint32_t stream, uint32_t rep,
                    uint32_t i) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {i >> 1, rep, stream, 0u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double U = (i & 1u) ? orc_u53(w[2], w[3]) : orc_u53(w[0], w[1]);
  int lo = 1, hi = K;
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (T[mid - 1] >= U)
      hi = mid;
    else
      lo = mid + 1;
  }
  return (int64_t)lo;
}

/* MLE (eq. 2 with the finite sums): mu(g) = -Z'/Z is the mean of ln X under */
/* the law, strictly decreasing from ln K (g -> -inf) to 0 (g -> +inf), so   */
/* the root of mu(g) = m is unique when 0 < m < ln K.  Newton with the same  */
/* bisection safeguard as orc_mle, on the bracket [-64, 64]; no root in the  */
/* bracket (e.g. every value equal to K) returns the bracket end, flagged    */
/* NOCONV.  The iteration stops after a step of at most 2^-40 max(|g|, 1)    */
/* and returns the next iterate: Newton converges quadratically, so that    */
/* iterate sits at the rounding noise of mu, while a tighter threshold can  */
/* lie below that noise when |g| < 1 and never be met.                      */
double orc_tz_mle(double m, int K, uint32_t *flags) {
  orc_iters = 0;
  double lo = -64.0, hi = 64.0;
  double z[3];
  orc_tz_norm3(hi, K, z);
  if (!(m > -z[1] / z[0])) { /* m at or below mu(64): the root is above 64 */
    *flags |= ORC_FLAG_NOCONV;
    return hi;
  }
  orc_tz_norm3(lo, K, z);
  if (!(m < -z[1] / z[0])) { /* m at or above mu(-64) */
    *flags |= ORC_FLAG_NOCONV;
    return lo;
  }
  double a = 1.0 + 1.0 / m;
  if (!(a > lo && a < hi)) a = 0.0;
  double g_last = 0.0;
  for (int it = 0; it < ORC_MLE_CAP; ++it) {
    orc_iters = it + 1;
    orc_tz_norm3(a, K, z);
    double r1 = z[1] / z[0];
    double gval = -r1 - m;
    if (gval == 0.0) return a;
    g_last = gval;
    if (gval > 0.0)
      lo = a;
    else
      hi = a;
    double gp = -(z[2] / z[0] - r1 * r1);
    double an = a - gval / gp;
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= ORC_FLAG_BISECT;
    }
    double scale = fabs(a) > 1.0 ? fabs(a) : 1.0;
    if (fabs(an - a) <= 0x1p-40 * scale) return an;
    a = an;
  }
  /* a residual within the rounding noise of mu is a root (as orc_hz_mle) */
  if (!(fabs(g_last) <= 0x1p-44 * m)) *flags |= ORC_FLAG_NOCONV;
  return a;
}

/* KS distance (eq. 3) of a sorted sample under the truncated law at g, by  */
/* the same reduction to distinct values as ks_sorted, F(t) = 1 - suf[t]/Z. */
static double tz_ks_sorted(const int64_t *xs, int64_t n, double g, int K) {
  double *suf = (double *)malloc(sizeof(double) * (size_t)(K + 1));
  tz_suffix(g, K, suf);
  const double z = suf[0], dn = (double)n;
  double D = 0.0;
  int64_t i = 0;
  while (i < n) {
    int64_t v = xs[i];
    int64_t below = i;
    while (i < n && xs[i] == v) ++i;
    int64_t upto = i;
    double Fv = 1.0 - suf[v] / z;
    double Fv1 = 1.0 - suf[v - 1] / z;
    if (v - 1 == 0) Fv1 = 0.0;
    double d1 = fabs((double)upto / dn - Fv);
    double d2 = fabs((double)below / dn - Fv1);
    if (d1 > D) D = d1;
    if (d2 > D) D = d2;
  }
  free(suf);
  return D;
}

static void tz_fit_sorted(const int64_t *xs, int64_t n, int K, double *S, double *ahat,
                          double *D, uint32_t *flags) {
  double s = neumaier_sum_log(xs, n);
  if (s == 0.0) {
    s = log(2.0);
    *flags |= ORC_FLAG_ALL_ONES;
  }
  double a = orc_tz_mle(s / (double)n, K, flags);
  *S = s;
  *ahat = a;
  *D = tz_ks_sorted(xs, n, a, K);
}

int orc_tz_fit(const int64_t *x, int64_t n, int K, double *S, double *g_hat, double *D,
               uint32_t *flags) {
  if (n < 1 || K < 2) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (x[i] < 1 || x[i] > K) return -1;
  int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!xs) return -1;
  memcpy(xs, x, sizeof(int64_t) * (size_t)n);
  qsort(xs, (size_t)n, sizeof(int64_t), cmp_i64);
  uint32_t f = 0;
  tz_fit_sorted(xs, n, K, S, g_hat, D, &f);
  *flags = f;
  free(xs);
  return 0;
}

typedef struct {
  double g;
  int K;
  int64_t n;
  uint64_t seed;
  uint32_t stream;
  int64_t rep_lo;
  const double *T;
  double *D, *ahat, *S;
  uint32_t *flags;
  uint64_t *fp;
  int64_t *xmax;
  int64_t begin, end;
} tz_job;

static void *tz_worker(void *arg) {
  tz_job *j = (tz_job *)arg;
  int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)j->n);
  for (int64_t r = j->begin; r < j->end; ++r) {
    uint32_t rep = (uint32_t)(j->rep_lo + r);
    uint32_t f = 0;
    uint64_t h = 0;
    for (int64_t i = 0; i < j->n; ++i) {
      x[i] = orc_tz_draw(j->T, j->K, j->seed, j->stream, rep, (uint32_t)i);
      h += mix64((uint64_t)x[i]);
    }
    qsort(x, (size_t)j->n, sizeof(int64_t), cmp_i64);
    double s, a, d;
    tz_fit_sorted(x, j->n, j->K, &s, &a, &d, &f);
    if (j->D) j->D[r] = d;
    if (j->ahat) j->ahat[r] = a;
    if (j->S) j->S[r] = s;
    if (j->flags) j->flags[r] = f;
    if (j->fp) j->fp[r] = h;
    if (j->xmax) j->xmax[r] = x[j->n - 1];
  }
  free(x);
  return NULL;
}

int orc_tz_simulate(double g, int K, int64_t n, uint64_t seed, uint32_t stream, int64_t rep_lo,
                    int64_t count, double *D, double *g_hat, double *S, uint32_t *flags,
                    uint64_t *fp, int64_t *xmax, int nthreads) {
  if (n < 1 || count < 0 || K < 2 || !isfinite(g)) return -1;
  double *T = (double *)malloc(sizeof(double) * (size_t)K);
  if (!T || orc_tz_cdf_table(g, K, T) != 0) {
    free(T);
    return -1;
  }
  int nt = resolve_threads(nthreads);
  if (nt > count) nt = count > 0 ? (int)count : 1;
  tz_job *jobs = (tz_job *)calloc((size_t)nt, sizeof(tz_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; ++t) {
    tz_job *j = &jobs[t];
    j->g = g;
    j->K = K;
    j->n = n;
    j->seed = seed;
    j->stream = stream;
    j->rep_lo = rep_lo;
    j->T = T;
    j->D = D;
    j->ahat = g_hat;
    j->S = S;
    j->flags = flags;
    j->fp = fp;
    j->xmax = xmax;
    j->begin = count * t / nt;
    j->end = count * (t + 1) / nt;
    if (nt == 1)
      tz_worker(j);
    else
      pthread_create(&th[t], NULL, tz_worker, j);
  }
  if (nt > 1)
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free(T);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The law with a lower cutoff xmin >= 1 (the practice the paper cites for   */
/* fitting power laws to data, Sect. 1; the paper itself fixes xmin = 1):    */
/*   p(k) = k^-alpha / zeta(alpha, xmin),  k >= xmin,                        */
/*   F(t) = 1 - zeta(alpha, t+1) / zeta(alpha, xmin) for t >= xmin, else 0.  */
/* MLE (eq. 2 with the Hurwitz zeta): -zeta'(a,xmin)/zeta(a,xmin) = mean     */
/* ln x over the values >= xmin.  mu(a) = -zeta'(a,xmin)/zeta(a,xmin) is    */
/* E_a[ln X], which decreases from +inf (a -> 1) to ln xmin (a -> inf), so a  */
/* root exists exactly when some value exceeds xmin.  If every value equals   */
/* xmin, one of them is counted as xmin + 1 (the all-ones rule of the pure    */
/* law, where xmin = 1).  xmin = 1 is the pure law and uses its functions.   */
/* ------------------------------------------------------------------------ */
void orc_hz_cdf_table(double alpha, int64_t xmin, double *T) {
  const double r = (double)xmin; /* both sums scaled by xmin^alpha */
  const double z = hurwitz0_rel(alpha, r, r);
  for (int j = 1; j <= ORC_TABLE_H; ++j)
    T[j - 1] = 1.0 - hurwitz0_rel(alpha, (double)(xmin + j), r) / z;
}

/* Tail of the law with cutoff: k >= m = xmin + H, the same floored-Pareto   */
/* rejection sampler as orc_tail_draw with its start moved to m.             */
static int64_t hz_tail_draw(double alpha, int64_t xmin, uint64_t seed, uint32_t stream,
                            uint32_t rep, uint32_t i, uint32_t *flags) {
  const double beta = alpha - 1.0;
  const double m = (double)(xmin + ORC_TABLE_H);
  const double gm = tail_g(beta, m);
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const __float128 two63 = 9223372036854775808.0Q;
  for (uint32_t attempt = 0; attempt < 0x7fffffffu; ++attempt) {
    uint32_t ctr[4] = {i, rep, stream, 0x80000000u | attempt};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double V = orc_u53(w[0], w[1]);
    double W = orc_u53(w[2], w[3]);
    __float128 Y = (__float128)m * expq(-logq((__float128)V) / (__float128)beta);
    if (Y >= two63) {
      *flags |= ORC_FLAG_TAIL_CAPPED;
      continue;
    }
    int64_t X = (int64_t)floorq(Y);
    if (W * gm <= tail_g(beta, (double)X)) return X;
  }
  return xmin + ORC_TABLE_H; /* unreachable in practice */
}

int64_t orc_hz_draw(double alpha, int64_t xmin, const double *T, uint64_t seed,
                    uint32_t stream, uint32_t rep, uint32_t i, uint32_t *flags) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {i >> 1, rep, stream, 0u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double U = (i & 1u) ? orc_u53(w[2], w[3]) : orc_u53(w[0], w[1]);
  if (U > T[ORC_TABLE_H - 1]) return hz_tail_draw(alpha, xmin, seed, stream, rep, i, flags);
  int lo = 1, hi = ORC_TABLE_H;
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (T[mid - 1] >= U)
      hi = mid;
    else
      lo = mid + 1;
  }
  return xmin - 1 + (int64_t)lo;
}

/* Newton-Raphson on g(a) = mu(a) - m in the bracket [1 + 2^-20, 64], as     */
/* orc_mle; stops after a step of at most 2^-40 a (with a large cutoff the   */
/* variance of ln X is small and mu is known to a few ulps only, so a        */
/* tighter test can lie below the noise).  With a large cutoff a sample      */
/* close to xmin can have its root above 64 (mu(64) - ln xmin is only about  */
/* 64/xmin^2 ... 1/xmin): then NOCONV and the bracket end 64.                */
double orc_hz_mle(double m, int64_t xmin, uint32_t *flags) {
  if (xmin == 1) return orc_mle(m, flags);
  orc_iters = 0;
  const double q = (double)xmin;
  double lo = 1.0 + 0x1p-20, hi = 64.0;
  {
    double z[3];
    orc_hurwitz3_scaled(hi, q, q, z); /* scaled by q^s: q^-64 underflows from q of about 6.5e4 */
    if (!(m > -z[1] / z[0])) { /* m at or below mu(64): the root is above 64 */
      *flags |= ORC_FLAG_NOCONV;
      return hi;
    }
  }
  double a = 1.0 + 1.0 / (m - log(q - 0.5)); /* continuous Pareto from xmin - 1/2 */
  if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
  double g_last = 0.0;
  for (int it = 0; it < ORC_MLE_CAP; ++it) {
    orc_iters = it + 1;
    double z[3];
    orc_hurwitz3_scaled(a, q, q, z);
    double r1 = z[1] / z[0];
    double g = -r1 - m;
    if (g == 0.0) return a;
    g_last = g;
    if (g > 0.0)
      lo = a;
    else
      hi = a;
    double gp = -(z[2] / z[0] - r1 * r1);
    double an = a - g / gp;
    if (!(an >= lo && an <= hi)) {
      an = 0.5 * (lo + hi);
      *flags |= ORC_FLAG_BISECT;
    }
    if (fabs(an - a) <= 0x1p-40 * a) return an;
    a = an;
  }
  /* Reading: eq. 2 is solved to FP64 precision.  Near the edge m -> ln xmin */
  /* it fixes the root only to about eps m / Var(ln X), coarser than the      */
  /* step test; a last residual within the rounding noise of mu is a root,    */
  /* not a failure to converge.                                               */
  if (!(fabs(g_last) <= 0x1p-44 * m)) *flags |= ORC_FLAG_NOCONV;
  return a;
}

/* D over the sorted values (all >= xmin): as ks_sorted with zeta(a, xmin)   */
/* as the normaliser and F(xmin - 1) = 0.                                    */
static double hz_ks_sorted(const int64_t *xs, int64_t n, double a, int64_t xmin) {
  const double r = (double)xmin; /* every sum scaled by xmin^a */
  const double z = hurwitz0_rel(a, r, r);
  const double dn = (double)n;
  double D = 0.0;
  int64_t i = 0;
  while (i < n) {
    int64_t v = xs[i];
    int64_t below = i;
    while (i < n && xs[i] == v) ++i;
    int64_t upto = i;
    double Fv = 1.0 - hurwitz0_rel(a, (double)v + 1.0, r) / z;
    double Fv1 = (v - 1 < xmin) ? 0.0 : 1.0 - hurwitz0_rel(a, (double)v, r) / z;
    double d1 = fabs((double)upto / dn - Fv);
    double d2 = fabs((double)below / dn - Fv1);
    if (d1 > D) D = d1;
    if (d2 > D) D = d2;
  }
  return D;
}

/* xs sorted ascending, every value >= xmin. */
static void hz_fit_sorted(const int64_t *xs, int64_t n, int64_t xmin, double *S, double *ahat,
                          double *D, uint32_t *flags) {
  if (xmin == 1) {
    fit_sorted(xs, n, S, ahat, D, flags);
    return;
  }
  double s;
  if (xs[n - 1] == xmin) { /* every value at the cutoff: count one as xmin + 1 */
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(tmp, xs, sizeof(int64_t) * (size_t)n);
    tmp[n - 1] = xmin + 1;
    s = neumaier_sum_log(tmp, n);
    free(tmp);
    *flags |= ORC_FLAG_ALL_ONES;
  } else {
    s = neumaier_sum_log(xs, n);
  }
  double a = orc_hz_mle(s / (double)n, xmin, flags);
  *S = s;
  *ahat = a;
  *D = hz_ks_sorted(xs, n, a, xmin);
}

int orc_hz_fit(const int64_t *x, int64_t n, int64_t xmin, int64_t *n_tail, double *S,
               double *alpha_hat, double *D, uint32_t *flags) {
  if (n < 1 || xmin < 1) return -1;
  int64_t *xs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!xs) return -1;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (x[i] < 1) {
      free(xs);
      return -1;
    }
    if (x[i] >= xmin) xs[m++] = x[i];
  }
  *n_tail = m;
  if (m == 0) {
    free(xs);
    return -2;
  }
  qsort(xs, (size_t)m, sizeof(int64_t), cmp_i64);
  uint32_t f = 0;
  hz_fit_sorted(xs, m, xmin, S, alpha_hat, D, &f);
  *flags = f;
  free(xs);
  return 0;
}

/* The KS-minimising choice of xmin: fit the values >= xmin for every        */
/* candidate and keep the one with the smallest D (the first on ties).       */
/* Candidates with no value at or above them get D = +inf.  Returns the     */
/* index of the chosen candidate, or -1 on invalid input.                    */
int orc_hz_scan(const int64_t *x, int64_t n, const int64_t *xmins, int n_xmin,
                double *alpha_hat, double *D, int64_t *n_tail, uint32_t *flags) {
  int best = -1;
  for (int c = 0; c < n_xmin; ++c) {
    double s;
    int rc = orc_hz_fit(x, n, xmins[c], &n_tail[c], &s, &alpha_hat[c], &D[c], &flags[c]);
    if (rc == -1) return -1;
    if (rc == -2) {
      alpha_hat[c] = 0.0;
      D[c] = INFINITY;
      flags[c] = 0;
      continue;
    }
    if (best < 0 || D[c] < D[best]) best = c;
  }
  return best;
}

typedef struct {
  double alpha;
  int64_t xmin, n;
  uint64_t seed;
  uint32_t stream;
  int64_t rep_lo;
  const double *T;
  double *D, *ahat, *S;
  uint32_t *flags;
  uint64_t *fp;
  int64_t *xmax;
  int64_t begin, end;
} hz_job;

static void *hz_worker(void *arg) {
  hz_job *j = (hz_job *)arg;
  int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (size_t)j->n);
  for (int64_t r = j->begin; r < j->end; ++r) {
    uint32_t rep = (uint32_t)(j->rep_lo + r);
    uint32_t f = 0;
    uint64_t h = 0;
    for (int64_t i = 0; i < j->n; ++i) {
      x[i] = orc_hz_draw(j->alpha, j->xmin, j->T, j->seed, j->stream, rep, (uint32_t)i, &f);
      h += mix64((uint64_t)x[i]);
    }
    qsort(x, (size_t)j->n, sizeof(int64_t), cmp_i64);
    double s, a, d;
    hz_fit_sorted(x, j->n, j->xmin, &s, &a, &d, &f);
    if (j->D) j->D[r] = d;
    if (j->ahat) j->ahat[r] = a;
    if (j->S) j->S[r] = s;
    if (j->flags) j->flags[r] = f;
    if (j->fp) j->fp[r] = h;
    if (j->xmax) j->xmax[r] = x[j->n - 1];
  }
  free(x);
  return NULL;
}

int orc_hz_simulate(double alpha, int64_t xmin, int64_t n, uint64_t seed, uint32_t stream,
                    int64_t rep_lo, int64_t count, double *D, double *alpha_hat, double *S,
                    uint32_t *flags, uint64_t *fp, int64_t *xmax, int nthreads) {
  if (n < 1 || count < 0 || xmin < 1 || !(alpha > 1.0)) return -1;
  double *T = (double *)malloc(sizeof(double) * ORC_TABLE_H);
  if (!T) return -1;
  orc_hz_cdf_table(alpha, xmin, T);
  int nt = resolve_threads(nthreads);
  if (nt > count) nt = count > 0 ? (int)count : 1;
  hz_job *jobs = (hz_job *)calloc((size_t)nt, sizeof(hz_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
  for (int t = 0; t < nt; ++t) {
    hz_job *j = &jobs[t];
    j->alpha = alpha;
    j->xmin = xmin;
    j->n = n;
    j->seed = seed;
    j->stream = stream;
    j->rep_lo = rep_lo;
    j->T = T;
    j->D = D;
    j->ahat = alpha_hat;
    j->S = S;
    j->flags = flags;
    j->fp = fp;
    j->xmax = xmax;
    j->begin = count * t / nt;
    j->end = count * (t + 1) / nt;
    if (nt == 1)
      hz_worker(j);
    else
      pthread_create(&th[t], NULL, hz_worker, j);
  }
  if (nt > 1)
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free(T);
  return 0;
}
