/*
 * zpl.h -- C ABI of libzpl, the MI355X (gfx950) implementation of the Monte
 * Carlo Kolmogorov-Smirnov method for the discrete power law of
 * E. Rappos and S. Robert, "Using GPU Simulation to Accurately Fit to the
 * Power-Law Distribution" (2013), for the pure (untruncated) law with xmin = 1.
 *
 * The method (Sect. 1-4 of the paper):
 *   eq. (1)  p(k) = k^-alpha / zeta(alpha),  k = 1, 2, ...
 *   eq. (2)  alpha_hat solves zeta'(a)/zeta(a) = -(1/N) sum_i ln x_i   (MLE)
 *   eq. (3)  D = sup_x |F(x; alpha_hat) - S_N(x)|                      (KS)
 * Critical values of D depend on N and alpha_hat because alpha is estimated
 * from the data, so they are obtained by simulation (Sect. 3): draw N values
 * at alpha, refit alpha by MLE, compute D, repeat, and read order statistics
 * of the simulated D.  Sect. 4 recommends a bespoke cutoff simulated at the
 * sample's own (N, alpha_hat); zpl_bootstrap_pvalue computes it as a p-value.
 *
 * Conventions this library fixes where the paper leaves a choice:
 *   - Random numbers: Philox4x32-10 with key = seed (low word first) and
 *     counter = (j, replicate, stream, 0) for draws 2j and 2j+1 (words 0-1
 *     and 2-3); tail proposals use counter (i, replicate, stream,
 *     0x80000000 | attempt).  Every draw is a pure function of (seed,
 *     stream, replicate, index): results never depend on launch shape.
 *   - U = ((w_hi:w_lo >> 11) | 1) * 2^-53.  x = min{k <= 4096 : F(k) >= U}
 *     (the paper's ">=" rule) when U <= F(4096); otherwise x comes from a
 *     rejection sampler on k >= 4097 conditioned on x < 2^63.
 *   - If every draw is 1, S = sum ln x is taken as ln 2 (the paper's rule).
 *   - alpha_hat is solved to full double precision on [1 + 2^-20, 64].
 *   - Quantile q = num/den of R values is the ascending order statistic at
 *     0-based index floor(R * num / den) (the paper's integer index rule).
 *   - p-value = #{b : D_b >= D_obs} / B.
 *
 * Memory: "host" pointers are ordinary CPU memory; "device" pointers are HIP
 * device memory on the context's GPU (e.g. a torch tensor's data_ptr()).  The
 * caller owns every buffer it passes; the library reads or writes them only
 * until the call returns (host buffers) or until the given stream reaches the
 * end of the work the call enqueued (device buffers), and never frees them.
 * The context owns all scratch memory.  A stream argument is a hipStream_t
 * (NULL = the null stream); calls that return host results synchronise it.
 *
 * Errors: every function returns a zpl_status; nothing is thrown across the
 * ABI.  On failure zpl_last_error() describes the error (per thread, valid
 * until the next call on that thread).  A context is not thread-safe: calls
 * on one context must be serialised by the caller, and because the calls
 * share the context's scratch, work enqueued by one call must not overlap on
 * the device with another's (use one stream per context, or synchronise
 * before switching streams).
 */
#ifndef ZPL_H
#define ZPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t zpl_status;
#define ZPL_OK 0
#define ZPL_EINVAL (-1)   /* invalid argument (n < 1, x < 1, alpha <= 1, ...) */
#define ZPL_ENOMEM (-2)   /* device memory or the context's budget exhausted   */
#define ZPL_EDEVICE (-3)  /* HIP runtime or kernel error                        */
#define ZPL_ENOCONV (-4)  /* the MLE solver did not converge (fit only)         */
#define ZPL_EBUSY (-5)    /* serving: not admissible now, retry later           */
#define ZPL_ENOTFOUND (-6) /* serving: unknown ticket                          */

/* Per-replicate / per-fit flags. */
#define ZPL_FLAG_ALL_ONES 1u    /* every value was 1 (at xmin); one counted as 2 (xmin + 1) */
#define ZPL_FLAG_TAIL_CAPPED 2u /* a tail proposal >= 2^63 was redrawn            */
#define ZPL_FLAG_BISECT 4u      /* the MLE solver took a bisection step (info)    */
#define ZPL_FLAG_NOCONV 8u      /* no MLE root in the bracket, or the iteration cap with the residual of eq. 2 above FP64 noise */

typedef struct zpl_ctx zpl_ctx;

/* One (alpha, n) cell of a critical-value table (Sect. 3; Table 1 for the
 * pure law, Tables 2-6 for the truncated one): R replicates of n draws at
 * exponent alpha, random stream (seed, stream).  Replicate r of the cell is
 * the same whatever else is computed alongside it.
 *   kmax = 0: the pure law of eq. (1) on k >= 1; alpha must lie in
 *             [1.01, 64] (closer to 1 the law puts so much mass at or above
 *             2^63 that the capped tail sampler slows down).
 *   kmax = K in 2..4096: the truncated law p(k) = k^-alpha / sum_{j<=K} j^-alpha
 *             on k = 1..K (Sect. 1 with a finite upper limit); alpha may be
 *             any value in [-64, 64], and alpha_hat is solved on [-64, 64]
 *             (ZPL_FLAG_NOCONV and the bracket end when the sample's mean log
 *             has no root there, e.g. every value equal to K).
 *   xmin      lower cutoff of the pure law (0 or 1: none; kmax must be 0
 *             otherwise; at most 2^40): p(k) = k^-alpha / zeta(alpha, xmin) on
 *             k >= xmin, the law used when a power law is fitted to the upper
 *             part of data (the practice the paper cites; its own tables have
 *             xmin = 1).  alpha_hat solves eq. (2) with the Hurwitz zeta on
 *             [1 + 2^-20, 64] (ZPL_FLAG_NOCONV and 64 when the root lies
 *             above); D is eq. (3) with F(t) = 1 - zeta(a, t+1)/zeta(a, xmin).
 *             If every value equals xmin, one is counted as xmin + 1 (the
 *             all-ones rule) and ZPL_FLAG_ALL_ONES is set.  Such cells run in
 *             the heavy form. */
typedef struct zpl_cell {
  double alpha;
  int64_t n;
  int64_t replicates;
  uint64_t seed;
  uint32_t stream;
  uint32_t kmax;
  int64_t xmin;
} zpl_cell;

/* Launch form of zpl_simulate_cells. */
#define ZPL_LAUNCH_BATCHED 0 /* one persistent launch over every cell (default) */
#define ZPL_LAUNCH_PLAIN 1   /* one launch per cell                              */

/* Per-cell execution form (the planner's choice unless forced). */
#define ZPL_FORM_AUTO 0
#define ZPL_FORM_LANE 1  /* one replicate per lane                     */
#define ZPL_FORM_WAVE 2  /* one replicate per wave, finishes per lane  */
#define ZPL_FORM_HEAVY 3 /* one replicate per wave, global overflow    */

typedef struct zpl_sim_opts {
  int32_t launch;    /* ZPL_LAUNCH_*                                     */
  int32_t form;      /* ZPL_FORM_*: force one form for every cell         */
  int32_t use_graph; /* 1: capture the batched launch in a hipGraph and
                        replay it when the same cell list is simulated
                        again                                            */
  int32_t reserved;  /* must be 0 */
} zpl_sim_opts;

/* Create a context on HIP device `device`.  mem_budget_bytes caps the
 * device scratch the context may hold (0 = 64 GiB). */
zpl_status zpl_create(zpl_ctx **out, int32_t device, uint64_t mem_budget_bytes);

/* Destroy a context and free its device memory.  NULL is ignored. */
void zpl_destroy(zpl_ctx *ctx);

/* Description of the last error on the calling thread ("" if none). */
const char *zpl_last_error(void);

/* Simulate critical-value cells (Sect. 3 and 4; Table 1 is such a table).
 *   cells[n_cells]           host; alpha in [1.01, 64], 1 <= n <= 2^31,
 *                            1 <= replicates <= 2^32.
 *   q_num[n_q], q_den[n_q]   host; quantile num/den with num < den.
 *   quantiles                host [n_cells * n_q] (row per cell) or NULL.
 *   d_out, alpha_hat_out     device [sum of replicates] FP64, or NULL;
 *   flags_out                device [sum of replicates] uint32, or NULL;
 *   fingerprint_out          device [sum of replicates] uint64, or NULL:
 *                            sum over draws of splitmix64's finaliser of the
 *                            value, mod 2^64 (a multiset checksum).
 *   Replicate r of cell c is at index (sum of replicates of cells < c) + r.
 *   opts may be NULL (batched, automatic forms, no graph).
 * Returns after the stream has finished when quantiles != NULL. */
zpl_status zpl_simulate_cells(zpl_ctx *ctx, const zpl_cell *cells, int32_t n_cells,
                              const uint32_t *q_num, const uint32_t *q_den, int32_t n_q,
                              double *quantiles, double *d_out, double *alpha_hat_out,
                              uint32_t *flags_out, uint64_t *fingerprint_out,
                              const zpl_sim_opts *opts, void *stream);

/* A whole critical-value table as the paper builds its Tables 1-6 (Sect. 3):
 * every entry is the mean, over n_seeds independent runs, of the quantile
 * order statistic of `replicates` simulated D values (the paper: 10 runs of
 * 50,000 at each (N, gamma), quantiles .90/.95/.99/.999).
 *   gammas[n_gamma], ns[n_n]  host; the table's columns (exponent) and rows
 *                             (sample size N); each (gamma, N) must be a
 *                             valid zpl_cell with this kmax.
 *   kmax                      0 = pure law (Table 1), else K (Tables 2-6).
 *   run s of entry (i_n, i_g) is the cell {gammas[i_g], ns[i_n], replicates,
 *   seed0 + s, stream = i_n * n_gamma + i_g, kmax}, so every entry and run
 *   can be recomputed alone with zpl_simulate_cells.
 *   table_out   host [n_n * n_gamma * n_q], entry (i_n, i_g, q) at
 *               (i_n * n_gamma + i_g) * n_q + q: the runs' quantiles summed
 *               in run order in FP64, then divided by n_seeds.
 *   per_run_out host [n_n * n_gamma * n_seeds * n_q] or NULL: the quantile of
 *               each run, (i_n, i_g, s, q) at ((i_n * n_gamma + i_g) *
 *               n_seeds + s) * n_q + q.
 * The runs go through the batched persistent launch in groups of cells
 * sized to the context's budget.  1 <= n_seeds <= 1024.  Synchronises the
 * stream. */
zpl_status zpl_critical_table(zpl_ctx *ctx, const double *gammas, int32_t n_gamma,
                              const int64_t *ns, int32_t n_n, uint32_t kmax, int32_t n_seeds,
                              uint64_t seed0, int64_t replicates, const uint32_t *q_num,
                              const uint32_t *q_den, int32_t n_q, double *table_out,
                              double *per_run_out, void *stream);

/* --------------------------------------------------------------------------
 * Autotuning of the execution form (the batched launch of Sect. 3's
 * simulations over cells of uneven n).  Every form computes the same bits;
 * the choice only changes speed.  The lane form runs one replicate per lane
 * and suits short replicates with light tails; the wave form runs one
 * replicate per wavefront with per-lane finishes; the heavy form keeps large
 * values in global memory.  A tuning table holds the measured cost of each
 * form on a grid of (alpha, n); with one installed, the planner gives every
 * cell the cheapest form eligible there (cost interpolated bilinearly in
 * alpha and ln n) and orders the work units by measured cost.
 * ------------------------------------------------------------------------ */
typedef struct zpl_tune_entry {
  double alpha;
  int64_t n;
  double ns_per_replicate[3]; /* lane, wave, heavy form: nanoseconds per
                                 replicate with the whole device busy;
                                 negative = form not eligible there       */
} zpl_tune_entry;

/* Measure the grid alphas[n_alpha] x ns[n_n] (each strictly increasing;
 * alpha in [1.01, 64], n in [1, 2^20], at most 64 values per axis) on the
 * context's device and install the table in the context.  table_out (host,
 * [n_alpha * n_n], alpha-major: entry ia * n_n + in) receives it, or NULL.
 * Each eligible (point, form) runs a probe cell sized to give every compute
 * unit one unit of work, twice; the probes are synchronous on `stream`. */
zpl_status zpl_autotune(zpl_ctx *ctx, const double *alphas, int32_t n_alpha,
                        const int64_t *ns, int32_t n_n, zpl_tune_entry *table_out,
                        void *stream);

/* Install a saved table (host, `count` entries in zpl_autotune's layout);
 * count = 0 removes it (built-in rule).  ZPL_EINVAL if the entries do not
 * form an alpha-major grid with increasing axes and finite costs. */
zpl_status zpl_set_tuning(zpl_ctx *ctx, const zpl_tune_entry *table, int32_t count);

/* The planner's form for each cell (ZPL_FORM_LANE/WAVE/HEAVY into
 * forms_out[n_cells], host) under `table` (count = 0: the built-in rule).
 * Host-only: touches no device and needs no context. */
zpl_status zpl_plan_forms(const zpl_tune_entry *table, int32_t count, const zpl_cell *cells,
                          int32_t n_cells, int32_t *forms_out);

/* Per-kernel timing of simulations (HIP events on the call's stream).
 * zpl_set_timing(ctx, 1) makes every later non-graph zpl_simulate_cells
 * record events around its kernels; zpl_get_timing then waits for the last
 * such call and writes ms4[0..3] = milliseconds spent in the table build,
 * the lane/wave simulation launches, the heavy/escalation launch and the
 * quantile selection.  ZPL_EINVAL if no timed call happened. */
zpl_status zpl_set_timing(zpl_ctx *ctx, int32_t enable);
zpl_status zpl_get_timing(zpl_ctx *ctx, double *ms4);

/* Fit one dataset (Sect. 4 usage): alpha_hat from eq. (2) and D from eq. (3).
 *   x[n]  host (x_on_device = 0) or device (1) int64, every x >= 1.
 *   alpha_hat, D, flags  host outputs.
 * Returns ZPL_EINVAL for n < 1 or any x < 1, ZPL_ENOCONV (outputs still set)
 * if the solver hit its iteration cap.  Synchronises the stream. */
zpl_status zpl_fit(zpl_ctx *ctx, const int64_t *x, int64_t n, int32_t x_on_device,
                   double *alpha_hat, double *D, uint32_t *flags, void *stream);

/* zpl_fit under the truncated law on 1..kmax (2 <= kmax <= 4096; every x in
 * 1..kmax, else ZPL_EINVAL): alpha_hat on [-64, 64] from eq. (2) with the
 * finite sums, and D from eq. (3) with the truncated CDF.  ZPL_ENOCONV
 * (outputs still set) if the mean log has no root in the bracket. */
zpl_status zpl_fit_truncated(zpl_ctx *ctx, const int64_t *x, int64_t n, int32_t x_on_device,
                             uint32_t kmax, double *alpha_hat, double *D, uint32_t *flags,
                             void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): zpl_fit
 * (kmax = 0) or zpl_fit_truncated (kmax = K in 2..4096) of a device dataset
 * into device outputs.  The call enqueues one kernel on `stream` and returns:
 * it allocates nothing, copies nothing to the host and does not synchronise.
 *   x_dev[n]        device int64; 1 <= n <= 2^20 (ZPL_EINVAL above that).
 *   alpha_hat_dev, D_dev    device double[1];  flags_dev device uint32[1]
 *                   (ZPL_FLAG_*; ZPL_FLAG_NOCONV where zpl_fit would return
 *                   ZPL_ENOCONV).
 *   status_dev      device uint32[1]: 0, or 2 when some x is out of range
 *                   (below 1, or above kmax); then the other outputs are not
 *                   written.
 * Results are bit-identical to zpl_fit / zpl_fit_truncated on the same data.
 * Scratch: a fixed device array of 2^22 + 4096 int64 (32 MiB and 32 KiB) per
 * GPU, the library's own, held until the process ends and shared by every
 * call on that GPU; it keeps the last call's contents (nothing in it must
 * start at zero).  Calls whose work overlaps on one GPU (other streams, other
 * contexts on the same device) race on it: serialise them. */
zpl_status zpl_fit_noalloc(zpl_ctx *ctx, const int64_t *x_dev, int64_t n, uint32_t kmax,
                           double *alpha_hat_dev, double *D_dev, uint32_t *flags_dev,
                           uint32_t *status_dev, void *stream);

/* Bespoke cutoff of Sect. 4 as a parametric-bootstrap p-value: fit x, then
 * simulate B replicates of n draws at alpha_hat (random stream (seed,
 * stream_id)), refit each by MLE (the tables apply only to MLE fits), and
 * return p = #{b : D_b >= D_obs} / B with alpha_hat, D_obs and the fit's
 * flags.  Synchronises the stream. */
zpl_status zpl_bootstrap_pvalue(zpl_ctx *ctx, const int64_t *x, int64_t n,
                                int32_t x_on_device, int64_t B, uint64_t seed,
                                uint32_t stream_id, double *alpha_hat, double *D,
                                double *p_value, uint32_t *flags, void *stream);

/* --------------------------------------------------------------------------
 * Serving: parametric-bootstrap requests (zpl_bootstrap_pvalue's computation,
 * Sect. 4's bespoke cutoff) under continuous batching.  A scheduler thread
 * admits queued requests, oldest first, as active slots and device memory
 * free up; fits each admitted dataset (eq. 2 and eq. 3) once; and then runs
 * the bootstraps of every active request together: each simulation launch
 * holds a window of replicates of every active request, the windows sized so
 * that a launch is about one time slice of work shared equally between the
 * requests.  A request that arrives while a launch runs joins the next one,
 * so its work shares the device with the bootstraps already in flight and a
 * short request is not held behind a long one; a request completes as soon
 * as its last window has run.  A request's result is bit-identical to
 * zpl_bootstrap_pvalue on the same (x, B, seed, stream_id), whatever it
 * shares the launches with.
 * ------------------------------------------------------------------------ */
typedef struct zpl_serve_opts {
  uint64_t mem_budget_bytes; /* device memory of the active requests (0 = 8 GiB;
                                at most the context's budget): 8 bytes per
                                bootstrap replicate while active, plus the
                                fit's dataset and scratch while it runs      */
  int32_t max_batch;         /* active requests at once (0 = 256)             */
  int32_t max_queue;         /* queued requests before submit says BUSY (0 = 65536) */
  int32_t slice_us;          /* target work per simulation launch, microseconds
                                of the whole device (0 = 4000)               */
  int32_t reserved2;         /* must be 0                                      */
} zpl_serve_opts;

typedef struct zpl_serve_result {
  int32_t done;        /* 0: still queued or running; 1: fields below valid     */
  zpl_status status;   /* ZPL_OK, ZPL_EINVAL (some x < 1), ZPL_ENOCONV (alpha_hat
                          below 1.01, no bootstrap), ZPL_ENOMEM (the request
                          alone exceeds the budget), ZPL_EDEVICE             */
  double alpha_hat;    /* eq. (2)                                             */
  double D;            /* eq. (3)                                             */
  double p_value;      /* #{b : D_b >= D} / B                                 */
  uint32_t flags;      /* fit flags (ZPL_FLAG_*)                               */
  int32_t batch_size;  /* most requests that shared a simulation launch with it */
  double queue_ms;     /* submit -> admission                                  */
  double latency_ms;   /* submit -> results ready                              */
  int32_t launches;    /* simulation launches that ran its replicates          */
  int32_t reserved;
} zpl_serve_result;

/* Start the scheduler on this context (opts may be NULL).  The scheduler
 * uses its own internal context and stream; the caller may keep using ctx.
 * ZPL_EINVAL if the serving budget exceeds the context's. */
zpl_status zpl_serve_start(zpl_ctx *ctx, const zpl_serve_opts *opts);

/* Queue one request: x[n] int64 in host memory (x_on_device = 0) or device
 * memory (1), copied before the call returns (a device dataset to a device
 * buffer of the scheduler's, where it stays until its fit; such copies are
 * not charged to the budget while queued); B bootstrap replicates; random
 * stream (seed, stream_id).  *ticket identifies it.  ZPL_EBUSY when max_queue
 * requests are already waiting. */
zpl_status zpl_serve_submit(zpl_ctx *ctx, const int64_t *x, int64_t n, int32_t x_on_device,
                            int64_t B, uint64_t seed, uint32_t stream_id, uint64_t *ticket);

/* Result of a request, waiting up to wait_ms for it (0 = do not wait).  A
 * completed result is returned once; the ticket is then released.
 * ZPL_ENOTFOUND for unknown or already released tickets. */
zpl_status zpl_serve_poll(zpl_ctx *ctx, uint64_t ticket, int32_t wait_ms,
                          zpl_serve_result *res);

/* Finish the queued requests and stop the scheduler. */
zpl_status zpl_serve_stop(zpl_ctx *ctx);

/* Raw draws of replicates rep_lo .. rep_lo+count-1 of cell (alpha, kmax, xmin,
 * n, seed, stream_id) in draw order, for checking the sampler bit for bit
 * (alpha, kmax and xmin as in zpl_cell).
 *   x_out     device [count * n] int64;  flags_out device [count] uint32
 *             (ZPL_FLAG_TAIL_CAPPED per replicate).
 * Asynchronous on `stream`. */
zpl_status zpl_sample_draws(zpl_ctx *ctx, double alpha, uint32_t kmax, int64_t xmin, int64_t n,
                            uint64_t seed, uint32_t stream_id, int64_t rep_lo, int64_t count,
                            int64_t *x_out, uint32_t *flags_out, void *stream);

/* The FP64 CDF table the sampler searches: T[j-1] = F(xmin - 1 + j; alpha),
 * j = 1..4096 (the truncated law's for kmax > 0, with F(k) = 1 for k >= kmax;
 * xmin as in zpl_cell).
 *   T_out  device [4096].  Asynchronous on `stream`. */
zpl_status zpl_cdf_table(zpl_ctx *ctx, double alpha, uint32_t kmax, int64_t xmin, double *T_out,
                         void *stream);

/* --------------------------------------------------------------------------
 * Fitting the upper part of data (the practice the paper cites for power-law
 * fits; the paper's own method has xmin = 1): the law with lower cutoff xmin
 * is fitted to the values >= xmin only (eq. 2 and eq. 3 with the Hurwitz
 * zeta, as for a zpl_cell with that xmin), and xmin itself is chosen as the
 * candidate whose fit has the smallest D.
 * ------------------------------------------------------------------------ */

/* Fit for each candidate cutoff, one wavefront per candidate, in one launch.
 *   x[n]            host (x_on_device = 0) or device int64, every x >= 1
 *                   (values below a candidate are ignored for that candidate).
 *   xmins[n_xmin]   host; each in [1, 2^40]; 1 <= n_xmin <= 65536.
 *   alpha_hat, D, n_tail, flags   host [n_xmin]: the fit of the values >=
 *                   xmins[c] and their count; a candidate above every value
 *                   has n_tail = 0, D = +inf, alpha_hat = 0.
 *   best            host: index of the smallest D (the first on ties), or -1
 *                   when no candidate has a value at or above it.
 * ZPL_EINVAL for n < 1, n > 2^31, any x < 1 or a candidate out of range.
 * A candidate whose MLE root lies above 64 keeps ZPL_FLAG_NOCONV in its flags
 * (the call still succeeds).  Synchronises the stream. */
zpl_status zpl_fit_scan(zpl_ctx *ctx, const int64_t *x, int64_t n, int32_t x_on_device,
                        const int64_t *xmins, int32_t n_xmin, double *alpha_hat, double *D,
                        int64_t *n_tail, uint32_t *flags, int32_t *best, void *stream);

/* zpl_fit_scan with the one candidate xmin.  ZPL_EINVAL also when no value is
 * >= xmin; ZPL_ENOCONV (outputs still set) when the MLE root lies above 64. */
zpl_status zpl_fit_xmin(zpl_ctx *ctx, const int64_t *x, int64_t n, int32_t x_on_device,
                        int64_t xmin, double *alpha_hat, double *D, int64_t *n_tail,
                        uint32_t *flags, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ZPL_H */
