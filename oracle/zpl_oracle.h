/*
 * zpl_oracle.h -- declarations of the reference (oracle) implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and zpl_oracle.c form a plain, slow CPU
 * implementation in FP64 (quad precision for one integer floor only) of the Monte Carlo Kolmogorov-Smirnov critical-value
 * method of Rappos & Robert, "Using GPU Simulation to Accurately Fit to the
 * Power-Law Distribution" (2013), for the pure discrete power law (Zipf,
 * xmin = 1).  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, constant or table with
 * the GPU library: the only things both sides agree on are the published
 * definitions they each implement (Philox4x32-10, the paper's equations, and
 * the conventions written down in the design notes).
 */
#ifndef ZPL_ORACLE_H
#define ZPL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the FP64 CDF table used for inverse-CDF sampling: values 1..4096
 * are drawn by table search, larger values by the rejection tail. */
#define ORC_TABLE_H 4096

/* Per-replicate flags (same bit meaning as the library's). */
#define ORC_FLAG_ALL_ONES     1u  /* every draw was 1; S replaced by ln 2   */
#define ORC_FLAG_TAIL_CAPPED  2u  /* a tail proposal >= 2^63 was redrawn   */
#define ORC_FLAG_BISECT       4u  /* the MLE solver took a bisection step  */
#define ORC_FLAG_NOCONV       8u  /* the MLE solver found no root: its     */
                                   /* iteration cap with a residual of eq. 2 */
                                   /* above FP64 noise, or no root in the    */
                                   /* bracket                                */

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* 53-bit uniform in (0,1) from two 32-bit words: ((hi:lo >> 11) | 1) * 2^-53. */
double orc_u53(uint32_t hi, uint32_t lo);

/* Hurwitz zeta zeta(s,q) and its first two derivatives in s (s > 1, q >= 1). */
void orc_hurwitz3(double s, double q, double out[3]);

/* Riemann zeta(s), zeta'(s), zeta''(s). */
void orc_zeta3(double s, double out[3]);

/* CDF of the pure Zipf law at integer t >= 0. */
double orc_cdf(double alpha, int64_t t);

/* T[k-1] = F(k; alpha) for k = 1..H. */
void orc_cdf_table(double alpha, double *T, int H);

/* Draw i of replicate `rep` in stream `stream` under key `seed`.
 * T must be orc_cdf_table(alpha, T, ORC_TABLE_H).  *flags gets
 * ORC_FLAG_TAIL_CAPPED or'ed in when a capped proposal was redrawn. */
int64_t orc_draw(double alpha, const double *T, uint64_t seed, uint32_t stream,
                 uint32_t rep, uint32_t i, uint32_t *flags);

/* The tail sampler alone: the value draw i of replicate `rep` takes when its
 * uniform exceeds T[H] (rejection on k >= H+1, conditioned on k < 2^63). */
int64_t orc_tail_draw(double alpha, uint64_t seed, uint32_t stream, uint32_t rep,
                      uint32_t i, uint32_t *flags);

/* n draws (in draw order) of one replicate. */
void orc_sample(double alpha, const double *T, int64_t n, uint64_t seed,
                uint32_t stream, uint32_t rep, int64_t *x, uint32_t *flags);

/* MLE of alpha from the mean log m = S/n (eq. 2), Newton with bisection. */
double orc_mle(double m, uint32_t *flags);
/* Iterations the calling thread's last MLE solve (any law) took. */
int orc_mle_last_iters(void);

/* Fit one dataset: S = sum ln x (all-ones rule applied), alpha_hat, D.
 * Returns 0, or -1 if n < 1 or any x < 1. */
int orc_fit(const int64_t *x, int64_t n, double *S, double *alpha_hat,
            double *D, uint32_t *flags);

/* Simulate replicates rep_lo .. rep_lo+count-1 of one (alpha, n) cell.
 * Any output pointer may be NULL.  fp[] receives, per replicate, the sum
 * over draws of splitmix64's finaliser of the drawn value (mod 2^64), a
 * multiset fingerprint used to check histograms bit for bit;
 * xmax[] the largest draw.  nthreads <= 0 means all online CPUs. */
int orc_simulate(double alpha, int64_t n, uint64_t seed, uint32_t stream,
                 int64_t rep_lo, int64_t count, double *D, double *alpha_hat,
                 double *S, uint32_t *flags, uint64_t *fp, int64_t *xmax,
                 int nthreads);

/* Order statistic at 0-based index floor(R*num/den) of D[0..R). */
double orc_quantile(const double *D, int64_t R, uint32_t num, uint32_t den);

/* Parametric bootstrap p-value: fit x, then simulate B replicates at
 * (n, alpha_hat) in stream `stream`, p = #{D_b >= D_obs} / B. */
int orc_bootstrap_pvalue(const int64_t *x, int64_t n, int64_t B, uint64_t seed,
                         uint32_t stream, double *alpha_hat, double *D,
                         double *p, uint32_t *flags, int nthreads);

/* ---- Truncated law on 1..K (Sect. 1 with a finite upper limit; Tables 2-6):
 * p(k) = k^-g / Z_K(g), Z_K(g) = sum_{k=1..K} k^-g, any real g, K >= 2.
 * Same random-number layout as the pure law's body draws; no tail. */

/* Z_K(g), Z_K'(g), Z_K''(g) by direct summation. */
void orc_tz_norm3(double g, int K, double out[3]);

/* T[k-1] = F(k; g, K) for k = 1..K (T[K-1] = 1).  Returns -1 if K < 2. */
int orc_tz_cdf_table(double g, int K, double *T);

/* Draw i of replicate `rep`: min{k <= K : T[k] >= U}. */
int64_t orc_tz_draw(const double *T, int K, uint64_t seed, uint32_t stream, uint32_t rep,
                    uint32_t i);

/* MLE of g on [-64, 64] from the mean log m (eq. 2 with finite sums). */
double orc_tz_mle(double m, int K, uint32_t *flags);

/* Fit one dataset (every x in 1..K).  Returns -1 on invalid input. */
int orc_tz_fit(const int64_t *x, int64_t n, int K, double *S, double *g_hat, double *D,
               uint32_t *flags);

/* orc_simulate for the truncated law. */
int orc_tz_simulate(double g, int K, int64_t n, uint64_t seed, uint32_t stream, int64_t rep_lo,
                    int64_t count, double *D, double *g_hat, double *S, uint32_t *flags,
                    uint64_t *fp, int64_t *xmax, int nthreads);

/* ---- the law with a lower cutoff xmin >= 1: p(k) = k^-alpha / zeta(alpha, xmin), k >= xmin ---- */

/* T[j-1] = F(xmin + j - 1), j = 1..ORC_TABLE_H. */
void orc_hz_cdf_table(double alpha, int64_t xmin, double *T);

/* Draw i of replicate rep: xmin - 1 + min{j : T[j] >= U}, or the rejection
 * tail on k >= xmin + ORC_TABLE_H. */
int64_t orc_hz_draw(double alpha, int64_t xmin, const double *T, uint64_t seed,
                    uint32_t stream, uint32_t rep, uint32_t i, uint32_t *flags);

/* alpha_hat for mean ln x = m (NOCONV and 64 when m <= ln xmin). */
double orc_hz_mle(double m, int64_t xmin, uint32_t *flags);

/* Fit the values >= xmin of a dataset.  Returns -1 on invalid input (n < 1,
 * xmin < 1, some x < 1), -2 if no value is >= xmin. */
int orc_hz_fit(const int64_t *x, int64_t n, int64_t xmin, int64_t *n_tail, double *S,
               double *alpha_hat, double *D, uint32_t *flags);

/* Fit for every candidate xmin; returns the index of the smallest D (first
 * on ties), -1 on invalid input.  D = +inf for a candidate above every value. */
int orc_hz_scan(const int64_t *x, int64_t n, const int64_t *xmins, int n_xmin,
                double *alpha_hat, double *D, int64_t *n_tail, uint32_t *flags);

/* orc_simulate for the law with cutoff xmin. */
int orc_hz_simulate(double alpha, int64_t xmin, int64_t n, uint64_t seed, uint32_t stream,
                    int64_t rep_lo, int64_t count, double *D, double *alpha_hat, double *S,
                    uint32_t *flags, uint64_t *fp, int64_t *xmax, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
