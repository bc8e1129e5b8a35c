// zpl_api.cpp -- host runtime and C ABI of libzpl (see include/zpl.h).
//
// The runtime validates calls, plans each cell (execution form, work units),
// owns the device scratch of a context, enqueues the kernels of
// zpl_kernels.hip on the caller's stream, and optionally captures the batched
// launch of a cell list in a hipGraph that later calls replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/zpl.h"
#include "zpl_kernels.hpp"
#include "zpl_launch.hpp"
#include "zpl_math.hpp"

using namespace zpl;

namespace {

thread_local std::string g_err;

zpl_status fail(zpl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? ZPL_ENOMEM : ZPL_EDEVICE, "%s: %s (%s)", \
                  #expr, hipGetErrorString(e_), __func__);                            \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Host staging of the ln table for the planner (same values the device uses
// are not needed here: the planner only estimates tail probabilities).
struct HostLn {
  std::vector<double> v;
  HostLn() : v(kH + 2) {
    v[0] = 0.0;
    for (int k = 1; k <= kH + 1; ++k) v[k] = std::log((double)k);
  }
};
const HostLn& host_ln() {
  static HostLn h;
  return h;
}

// Smallest exponent simulated.  Below it the tail law's mass above 2^63 makes
// the capped rejection sampler take many attempts per draw.  (Fitted
// exponents are never below about 1.023: mean ln x < ln 2^63.)
constexpr double kMinAlpha = 1.01;
constexpr int64_t kMaxXmin = (int64_t)1 << 40;
// Datasets at least this long are fitted by a whole workgroup.
constexpr int64_t kFitBlockMin = 2048;
// Host datasets up to this many bytes go through pinned staging.
constexpr size_t kPinStageMax = (size_t)64 << 20;

// P(X > h) under exponent a: the pure law (K = 0) or the truncated law on
// 1..K (finite sums).
double tail_prob(double a, int h, uint32_t K = 0) {
  if (K > 0) {
    if ((uint32_t)h >= K) return 0.0;
    double z = 0.0, t = 0.0;
    for (int k = (int)K; k >= 1; --k) {
      const double w = std::exp(-a * host_ln().v[k]);
      z += w;
      if (k > h) t += w;
    }
    return t / z;
  }
  double suf[17];
  survival_head(a, host_ln().v.data(), suf);
  const double zt = h >= 16 ? survival_next(a, h, host_ln().v.data()) : suf[h];
  return zt / suf[0];
}

struct Tuning {
  std::vector<double> alphas;  // strictly increasing
  std::vector<int64_t> ns;     // strictly increasing
  std::vector<double> cost;    // [(ia * ns.size() + in) * 3 + form], < 0: not measured
  bool empty() const { return alphas.empty(); }
};

}  // namespace

struct Server;

struct zpl_ctx {
  Server* server = nullptr;
  int device = 0;
  int n_cu = 256;
  uint64_t budget = 0;
  uint64_t used = 0;
  double* ln = nullptr;
  // device address of the allocation-free fit's fixed scratch array on this
  // context's GPU (looked up once, at creation)
  int64_t* noalloc_scratch = nullptr;
  // scratch, grow-only
  // plan: the cells, then (simulation calls) the units, heavy units and the
  // quantile numerators and denominators, uploaded with one copy; ctr: the
  // work queues, escalation count and error word, cleared by the table
  // kernel, then the quantile results, so that error word and quantiles come
  // back with one copy (layout: PlanLayout)
  DevBuf plan, ctr, tables, guides, esc, list_v, list_c, wslots, heavy, dbuf, gather, fit_x,
      fit_ptrs, fit_ns, fit_out, fit_st, count, boot_d, scan;
  // pinned host staging
  void* pin = nullptr;
  size_t pin_bytes = 0;
  void* pin_x = nullptr;  // host datasets on their way to fit_x
  size_t pin_x_bytes = 0;
  // graph cache (one entry)
  bool graph_valid = false;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<char> graph_key;
  // The plan buffer is rewritten by every call; plan_gen counts the uploads,
  // and a replay re-uploads its plan when another call wrote the buffer
  // after it (graph_plan_gen).
  uint64_t plan_gen = 0, graph_plan_gen = 0;
  uint32_t esc_cap = 0;
  // optional per-kernel timing of the last non-graph simulation
  hipStream_t cap_stream = nullptr;  // graphs are captured here (never the null stream)
  bool timing = false;
  bool timed = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t err_off = 0;  // byte offset of the last simulation's error word in ctr
  Tuning tune;  // measured form costs (empty: built-in rule)
};

namespace {

zpl_status ensure(zpl_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return ZPL_OK;
  if (b.p) {
    HIP_TRY(hipDeviceSynchronize());  // in-flight work may still use it
    HIP_TRY(hipFree(b.p));
    c->used -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  // any cached graph may point at the freed buffer
  if (c->graph_valid) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_valid = false;
    c->graph_key.clear();
  }
  if (c->used + bytes > c->budget)
    return fail(ZPL_ENOMEM, "device scratch of %zu bytes exceeds the context budget (%llu of %llu used)",
                bytes, (unsigned long long)c->used, (unsigned long long)c->budget);
  HIP_TRY(hipMalloc(&b.p, bytes));
  b.bytes = bytes;
  c->used += bytes;
  return ZPL_OK;
}

// Size for a buffer on a latency path (dataset staging, fit scratch): the
// next power of two, at least 1 MiB, so that datasets of growing size do not
// reallocate (a reallocation synchronises the device) on most calls; sizes
// above 64 MiB are taken as they are.
size_t grow_size(size_t bytes) {
  if (bytes > ((size_t)64 << 20)) return bytes;
  size_t v = (size_t)1 << 20;
  while (v < bytes) v <<= 1;
  return v;
}

zpl_status ensure_pinned(zpl_ctx* c, size_t bytes) {
  if (c->pin_bytes >= bytes) return ZPL_OK;
  HIP_TRY(hipDeviceSynchronize());  // async copies may still read the old area
  if (c->pin) HIP_TRY(hipHostFree(c->pin));
  c->pin = nullptr;
  c->pin_bytes = 0;
  HIP_TRY(hipHostMalloc(&c->pin, bytes, hipHostMallocDefault));
  c->pin_bytes = bytes;
  return ZPL_OK;
}

#define ZPL_TRY(expr)             \
  do {                            \
    zpl_status s_ = (expr);       \
    if (s_ != ZPL_OK) return s_;  \
  } while (0)

// ---------------------------------------------------------------------------
// Tuning table: the measured cost (ns per replicate, whole device busy) of
// each execution form on a grid of (alpha, n).  With a table the planner
// picks the cheapest eligible form of every cell and orders the work units by
// measured cost; without one it uses the built-in rule below.  Every form
// gives the same bits, so a table changes speed only.
// ---------------------------------------------------------------------------

constexpr int kTuneMaxAxis = 64;

zpl_status parse_tuning(const zpl_tune_entry* e, int32_t count, Tuning& t) {
  t = Tuning();
  if (count == 0) return ZPL_OK;
  if (count < 0 || !e) return fail(ZPL_EINVAL, "tuning table: bad count or NULL entries");
  // alpha-major grid: the n axis is the run of entries sharing the first alpha
  int nn = 1;
  while (nn < count && e[nn].alpha == e[0].alpha) ++nn;
  if (count % nn != 0)
    return fail(ZPL_EINVAL, "tuning table: %d entries do not form an alpha x n grid", count);
  const int na = count / nn;
  if (na > kTuneMaxAxis || nn > kTuneMaxAxis)
    return fail(ZPL_EINVAL, "tuning table: at most %d values per axis", kTuneMaxAxis);
  for (int ia = 0; ia < na; ++ia) {
    const double a = e[ia * nn].alpha;
    if (!(a >= 1.0 && a <= 64.0)) return fail(ZPL_EINVAL, "tuning table: alpha %g outside (1, 64]", a);
    if (ia > 0 && !(a > t.alphas.back()))
      return fail(ZPL_EINVAL, "tuning table: alphas must increase");
    t.alphas.push_back(a);
  }
  for (int in = 0; in < nn; ++in) {
    const int64_t n = e[in].n;
    if (n < 1) return fail(ZPL_EINVAL, "tuning table: n must be >= 1");
    if (in > 0 && !(n > t.ns.back())) return fail(ZPL_EINVAL, "tuning table: n must increase");
    t.ns.push_back(n);
  }
  t.cost.resize((size_t)count * 3);
  for (int ia = 0; ia < na; ++ia)
    for (int in = 0; in < nn; ++in) {
      const zpl_tune_entry& x = e[ia * nn + in];
      if (x.alpha != t.alphas[ia] || x.n != t.ns[in])
        return fail(ZPL_EINVAL, "tuning table: entry %d is not (alpha %g, n %lld) of the grid",
                    ia * nn + in, t.alphas[ia], (long long)t.ns[in]);
      for (int f = 0; f < 3; ++f) {
        const double v = x.ns_per_replicate[f];
        if (!std::isfinite(v)) return fail(ZPL_EINVAL, "tuning table: cost not finite");
        t.cost[(size_t)(ia * nn + in) * 3 + f] = v;
      }
    }
  return ZPL_OK;
}

// Position of x on an increasing axis: segment i and weight w of axis[i+1]
// (clamped to the ends).
void axis_locate(const std::vector<double>& ax, double x, int& i, double& w) {
  const int m = (int)ax.size();
  if (m == 1 || x <= ax[0]) {
    i = 0;
    w = 0.0;
    return;
  }
  if (x >= ax[m - 1]) {
    i = m - 2;
    w = 1.0;
    return;
  }
  i = 0;
  while (ax[i + 1] < x) ++i;
  w = (x - ax[i]) / (ax[i + 1] - ax[i]);
}

// Cost per replicate of form f (0 lane, 1 wave, 2 heavy) at (alpha, n):
// bilinear in (alpha, ln n) on the grid, clamped in alpha and below the
// smallest n, proportional to n above the largest.  Negative when a grid
// corner that carries weight at the point has no measurement.
double tuned_cost(const Tuning& t, int f, double alpha, int64_t n) {
  std::vector<double> lns(t.ns.size());
  for (size_t k = 0; k < t.ns.size(); ++k) lns[k] = std::log((double)t.ns[k]);
  int ia, in;
  double wa, wn;
  axis_locate(t.alphas, alpha, ia, wa);
  axis_locate(lns, std::log((double)n), in, wn);
  const int nn = (int)t.ns.size();
  const int ia1 = std::min(ia + 1, (int)t.alphas.size() - 1), in1 = std::min(in + 1, nn - 1);
  const double c00 = t.cost[(size_t)(ia * nn + in) * 3 + f];
  const double c01 = t.cost[(size_t)(ia * nn + in1) * 3 + f];
  const double c10 = t.cost[(size_t)(ia1 * nn + in) * 3 + f];
  const double c11 = t.cost[(size_t)(ia1 * nn + in1) * 3 + f];
  const double w00 = (1 - wa) * (1 - wn), w01 = (1 - wa) * wn, w10 = wa * (1 - wn), w11 = wa * wn;
  // a corner that carries weight must have a measurement
  if ((w00 > 0 && c00 < 0) || (w01 > 0 && c01 < 0) || (w10 > 0 && c10 < 0) || (w11 > 0 && c11 < 0))
    return -1.0;
  double v = (w00 > 0 ? w00 * c00 : 0.0) + (w01 > 0 ? w01 * c01 : 0.0) +
             (w10 > 0 ? w10 * c10 : 0.0) + (w11 > 0 ? w11 * c11 : 0.0);
  if (n > t.ns.back()) v *= (double)n / (double)t.ns.back();
  return v;
}

// ---------------------------------------------------------------------------
// Planner: execution form per cell and the unit list.
// ---------------------------------------------------------------------------
struct Plan {
  std::vector<DevCell> cells;
  std::vector<Unit> units;    // lane and wave units (LPT order)
  std::vector<Unit> hunits;   // heavy units
  std::vector<int> cell_unit_begin, cell_unit_end;  // per cell range in `units`
  int64_t total_R = 0;
  int64_t max_n = 0;
  int64_t lw_R = 0;  // replicates in lane and wave cells
};

// Forms a tuned planner may pick: the lane form only where a replicate rarely
// overflows its per-lane list, the wave form only where the LDS overflow
// area almost surely holds a replicate's large values.
bool form_eligible(uint32_t m, double alpha, int64_t n, uint32_t K = 0) {
  if (m == kModeLane) {  // values above the column: kLaneCap slots in scratch
    if (n > 65535) return false;
    const double mu = (double)n * tail_prob(alpha, kHLB, K);
    return mu + 8.0 * std::sqrt(mu) + 8.0 <= (double)kLaneCap;
  }
  if (m == kModeWave) {
    const double mu = (double)n * tail_prob(alpha, kHW, K);
    return mu + 8.0 * std::sqrt(mu) + 8.0 <= (double)kCW;
  }
  return true;
}

// Estimated cost (ns per replicate, device busy) of a replicate of the
// truncated law on 1..K with n draws, in the lane or wave form: about 2.2 ps
// per draw and 19 ps per support value (sums of the MLE and the KS distance),
// measured on MI355X over the paper's sample sizes at K = 20 and K = 1000.
double trunc_cost(int64_t n, uint32_t K) { return 2.2e-3 * ((double)n + 8.6 * (double)K); }

// Time for one cell alone under form f (tuned cost v ns per replicate with
// the device busy): its work units (kBlock replicates per workgroup for the
// lane and wave forms, 8 for the heavy form, which fits two workgroups per
// compute unit) run in rounds of as many units as the device holds at once,
// and a unit takes v x (replicates the device holds at once).
double cell_makespan(int f, double v, int64_t R, int n_cu) {
  const double per = f == (int)kModeHeavy ? 8.0 : (double)kBlock;
  const double conc = f == (int)kModeHeavy ? 2.0 * n_cu : (double)n_cu;
  return std::ceil(std::ceil((double)R / per) / conc) * v * conc * per;
}

// Pure law with a tuning table: the eligible form of least cost per replicate, or,
// when `horizon` (ns) is given and that form alone would take longer than
// the horizon (a few thousand long replicates, as in a bootstrap, fill only
// a few workgroups), the form that finishes the cell soonest.  Otherwise
// (no table, or the truncated law): the lane form when a replicate's values
// above its column are few, else the wave form when its overflow area holds
// them, else the heavy form.
uint32_t choose_form(double alpha, int64_t n, const Tuning* t, uint32_t K = 0, int64_t R = 0,
                     int n_cu = 256, double horizon = -1.0, double* cost = nullptr) {
  if (cost) *cost = 0.0;
  if (K > 0) {
    // the table measures the pure law; the truncated law's cost is mostly
    // its finite sums (K terms per MLE step), which the heavy form runs one
    // replicate per wave: the built-in rule below, with an estimated cost
    if (cost && t && !t->empty()) *cost = trunc_cost(n, K) * (double)R;
  } else if (t && !t->empty()) {
    int best = -1, fast = -1;
    double bc = 0.0, bm = 0.0;
    for (int f = 0; f < 3; ++f) {
      if (!form_eligible((uint32_t)f, alpha, n, K)) continue;
      const double v = tuned_cost(*t, f, alpha, n);
      if (!(v >= 0.0)) continue;
      if (best < 0 || v < bc) {
        best = f;
        bc = v;
      }
      const double m = cell_makespan(f, v, R, n_cu);
      if (fast < 0 || m < bm) {
        fast = f;
        bm = m;
      }
    }
    if (best >= 0) {
      if (cost) *cost = bc * (double)R;
      if (horizon >= 0.0 && R > 0 && cell_makespan(best, bc, R, n_cu) > horizon) return (uint32_t)fast;
      return (uint32_t)best;
    }
  }
  if (n <= 65535 && (double)n * tail_prob(alpha, kHLB, K) <= 2.0) return kModeLane;
  if (form_eligible(kModeWave, alpha, n, K)) return kModeWave;
  return kModeHeavy;
}

// rlo (optional): cell i covers replicates rlo[i] .. rlo[i] + replicates - 1
// (a window of a longer cell, as the serving scheduler runs them); its
// outputs still start at the cell's prefix position in the per-replicate
// arrays.  Without it every cell covers replicates 0 .. replicates - 1.
zpl_status make_plan(const zpl_cell* cells, int n_cells, int form, Plan& P,
                     const Tuning* tune = nullptr, int n_cu = 256,
                     const int64_t* rlo = nullptr) {
  P = Plan();
  P.cells.resize(n_cells);
  P.cell_unit_begin.assign(n_cells, 0);
  P.cell_unit_end.assign(n_cells, 0);
  // the batch's work with every cell in its cheapest form: a cell that alone
  // would outlast it is given the form that finishes it soonest instead
  double horizon = -1.0;
  if (form == ZPL_FORM_AUTO && tune && !tune->empty()) {
    horizon = 0.0;
    for (int i = 0; i < n_cells; ++i) {
      const zpl_cell& z = cells[i];
      double c = 0.0;
      const bool valid = z.kmax == 0 ? (z.alpha >= kMinAlpha && z.alpha <= 64.0)
                                     : (z.kmax >= 2 && z.kmax <= (uint32_t)kH &&
                                        z.alpha >= -64.0 && z.alpha <= 64.0);
      // (invalid cells are rejected below; cutoff cells run in the heavy form)
      if (valid && z.n >= 1 && z.replicates >= 1 && (z.xmin == 0 || z.xmin == 1))
        (void)choose_form(z.alpha, z.n, tune, z.kmax, z.replicates, n_cu, -1.0, &c);
      horizon += c;
    }
  }
  for (int i = 0; i < n_cells; ++i) {
    const zpl_cell& z = cells[i];
    if (z.kmax == 0) {
      if (!(z.alpha >= kMinAlpha) || !(z.alpha <= 64.0))
        return fail(ZPL_EINVAL, "cell %d: alpha must be in [1.01, 64], got %g", i, z.alpha);
    } else {
      if (z.kmax < 2 || z.kmax > (uint32_t)kH)
        return fail(ZPL_EINVAL, "cell %d: kmax must be 0 or in [2, %d], got %u", i, kH, z.kmax);
      if (!(z.alpha >= -64.0) || !(z.alpha <= 64.0))
        return fail(ZPL_EINVAL, "cell %d: alpha must be in [-64, 64], got %g", i, z.alpha);
    }
    const int64_t xmin = z.xmin == 0 ? 1 : z.xmin;
    if (xmin < 1 || xmin > kMaxXmin)
      return fail(ZPL_EINVAL, "cell %d: xmin must be 0, 1 or in [2, 2^40], got %lld", i,
                  (long long)z.xmin);
    if (xmin > 1 && z.kmax != 0)
      return fail(ZPL_EINVAL, "cell %d: xmin > 1 needs kmax = 0 (the pure law)", i);
    if (z.n < 1 || z.n > ((int64_t)1 << 31))
      return fail(ZPL_EINVAL, "cell %d: n must be in [1, 2^31], got %lld", i, (long long)z.n);
    if (z.replicates < 1 || z.replicates > ((int64_t)1 << 32))
      return fail(ZPL_EINVAL, "cell %d: replicates must be in [1, 2^32], got %lld", i,
                  (long long)z.replicates);
    if (rlo && (rlo[i] < 0 || rlo[i] + z.replicates > ((int64_t)1 << 32)))
      return fail(ZPL_EINVAL, "cell %d: replicate window out of range", i);
    DevCell& d = P.cells[i];
    std::memset(&d, 0, sizeof d);
    d.alpha = z.alpha;
    d.n = z.n;
    d.R = z.replicates;
    d.out_off = P.total_R - (rlo ? rlo[i] : 0);  // output index = out_off + replicate
    d.k0 = (uint32_t)z.seed;
    d.k1 = (uint32_t)(z.seed >> 32);
    d.stream = z.stream;
    d.K = z.kmax;
    d.xmin = xmin;
    uint32_t m;
    switch (form) {
      case ZPL_FORM_LANE:
        m = kModeLane;
        if (z.n > 65535) return fail(ZPL_EINVAL, "cell %d: lane form needs n <= 65535", i);
        break;
      case ZPL_FORM_WAVE: m = kModeWave; break;
      case ZPL_FORM_HEAVY: m = kModeHeavy; break;
      default: m = choose_form(z.alpha, z.n, tune, z.kmax, z.replicates, n_cu, horizon);
    }
    // the lane and wave forms histogram values from 1; a cutoff law runs in
    // the heavy form, whose histogram and overflow list take any values
    if (xmin > 1) {
      if (form == ZPL_FORM_LANE || form == ZPL_FORM_WAVE)
        return fail(ZPL_EINVAL, "cell %d: a cell with xmin > 1 runs in the heavy form only", i);
      m = kModeHeavy;
    }
    d.mode = m;
    P.total_R += z.replicates;
    P.max_n = std::max(P.max_n, z.n);
    if (m != kModeHeavy) P.lw_R += z.replicates;
  }
  // units: kBlock replicates (one per lane, or 64 per wave) for lane/wave
  // cells, 8 replicates (2 per wave) for heavy cells.  The longest-first
  // order weighs a unit by how long it occupies its workgroup: per-replicate
  // cost (from the tuning table when there is one; the truncated law: draws
  // plus its K-term sums, see trunc_cost) times the replicates its busiest
  // wave runs one after another -- min(count, 64) in the wave form, one per
  // lane (64 in these units) in the lane form.  Weighing by count instead
  // sent each wave-form cell's last, partial unit to the end of the queue,
  // where it ran as long as a full one on an otherwise idle device.
  // Every unit of a cell but the last holds kBlock replicates, so a cell's
  // units take at most two weights: the order is built from at most two runs
  // of units per cell (sorted by weight, then cell; a run keeps ascending
  // replicates), not by sorting the units themselves.
  struct Run {
    double w;
    int cell;
    int64_t r_begin, r_end;  // units start at r_begin, r_begin + kBlock, ... < r_end
  };
  std::vector<Run> runs;
  size_t n_units = 0;
  for (int i = 0; i < n_cells; ++i) {
    const DevCell& d = P.cells[i];
    const int64_t r0 = rlo ? rlo[i] : 0;
    if (d.mode == kModeHeavy) {
      for (int64_t r = 0; r < d.R; r += 8) {
        Unit u;
        u.cell = i;
        u.r0 = r0 + r;
        u.count = (int32_t)std::min<int64_t>(8, d.R - r);
        P.hunits.push_back(u);
      }
      continue;
    }
    if (d.R <= 0) continue;
    double w = d.K ? (double)d.n + 8.6 * (double)d.K : (double)d.n;
    if (tune && !tune->empty()) {
      const double v = d.K ? trunc_cost(d.n, d.K) : tuned_cost(*tune, (int)d.mode, d.alpha, d.n);
      if (v > 0.0) w = v;
    }
    auto weight = [&](int64_t count) {
      return w * (d.mode == kModeLane ? 64.0 : (double)std::min<int64_t>(count, 64));
    };
    const int64_t r_last = (d.R - 1) / kBlock * kBlock;
    const double w_last = weight(d.R - r_last);
    if (r_last > 0 && weight(kBlock) != w_last) {
      runs.push_back({weight(kBlock), i, 0, r_last});
      runs.push_back({w_last, i, r_last, d.R});
    } else {
      runs.push_back({w_last, i, 0, d.R});
    }
    n_units += (size_t)((d.R + kBlock - 1) / kBlock);
  }
  // longest units first; ties by cell so a workgroup tends to keep its table
  std::sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) {
    if (a.w != b.w) return a.w > b.w;
    return a.cell < b.cell;
  });
  P.units.reserve(n_units);
  for (const Run& g : runs) {
    const DevCell& d = P.cells[g.cell];
    const int64_t r0 = rlo ? rlo[g.cell] : 0;
    for (int64_t r = g.r_begin; r < g.r_end; r += kBlock) {
      Unit u;
      u.cell = g.cell;
      u.r0 = r0 + r;
      u.count = (int32_t)std::min<int64_t>(kBlock, d.R - r);
      P.units.push_back(u);
    }
  }
  return ZPL_OK;
}

// Units of one cell, for plain launches: contiguous by construction below.
void plain_unit_order(Plan& P) {
  std::stable_sort(P.units.begin(), P.units.end(),
                   [](const Unit& a, const Unit& b) { return a.cell < b.cell; });
  for (size_t k = 0; k < P.units.size(); ++k) {
    const int c = P.units[k].cell;
    if (k == 0 || P.units[k - 1].cell != c) P.cell_unit_begin[c] = (int)k;
    P.cell_unit_end[c] = (int)k + 1;
  }
}

int64_t heavy_stride(int64_t max_n) {
  int64_t p2 = 1;
  while (p2 < max_n) p2 <<= 1;
  int64_t half = std::max<int64_t>(p2, 2 * ((int64_t)kHeavyHist + max_n));
  half = (half + 1) & ~(int64_t)1;
  return 2 * half;
}

// Byte offsets of a simulation call's parts in the plan and ctr buffers.
// plan: cells | units | heavy units | q_num | q_den, each part 256-byte
// aligned.  ctr (32-bit words): the work queues (nc + 8, rounded up to even),
// the escalation count (4), the error word (4), then the nc * n_q quantile
// results (doubles), so that [error word .. quantiles] is contiguous.
struct PlanLayout {
  size_t units = 0, hunits = 0, qnum = 0, qden = 0, plan_bytes = 0;
  int ctr_words = 0;           // words cleared before each run
  size_t esc = 0, err = 0, qout = 0, ctr_bytes = 0;
};

PlanLayout plan_layout(const Plan& P, int n_q) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t nc = P.cells.size();
  PlanLayout L;
  L.units = up(sizeof(DevCell) * nc);
  L.hunits = L.units + up(sizeof(Unit) * P.units.size());
  L.qnum = L.hunits + up(sizeof(Unit) * P.hunits.size());
  L.qden = L.qnum + up(sizeof(uint32_t) * (size_t)n_q);
  L.plan_bytes = L.qden + sizeof(uint32_t) * (size_t)n_q;
  const size_t qw = (nc + 8 + 1) & ~(size_t)1;
  L.esc = sizeof(uint32_t) * qw;
  L.err = L.esc + sizeof(uint32_t) * 4;
  L.qout = L.err + sizeof(uint32_t) * 4;
  L.ctr_words = (int)(qw + 8);
  L.ctr_bytes = L.qout + sizeof(double) * nc * (size_t)n_q;
  return L;
}

struct Launch {
  int sim_grid = 0;
  int heavy_grid = 0;
  int64_t hstride = 0;
  int64_t gcap = 0;
  int64_t maxR = 1;
  PlanLayout lay;
};

// Grows every scratch buffer the plan needs.
zpl_status prepare(zpl_ctx* c, const Plan& P, int n_q, bool need_dbuf, Launch& L) {
  const int nc = (int)P.cells.size();
  L.lay = plan_layout(P, n_q);
  ZPL_TRY(ensure(c, c->plan, L.lay.plan_bytes));
  ZPL_TRY(ensure(c, c->ctr, L.lay.ctr_bytes));
  c->err_off = L.lay.err;
  ZPL_TRY(ensure(c, c->tables, sizeof(double) * (size_t)kH * nc));
  ZPL_TRY(ensure(c, c->guides, sizeof(uint16_t) * (size_t)(kGuide + 1) * nc));
  // escalation list: a slot for every lane/wave replicate (each escalates at
  // most once), so it cannot overflow below 2^31 such replicates
  const uint32_t esc_cap =
      (uint32_t)std::min<int64_t>(std::max<int64_t>(P.lw_R, 64), (int64_t)1 << 31);
  ZPL_TRY(ensure(c, c->esc, sizeof(uint64_t) * esc_cap));
  c->esc_cap = esc_cap;
  const int sim_grid =
      (int)std::min<int64_t>((int64_t)P.units.size(), (int64_t)c->n_cu);
  L.sim_grid = sim_grid;
  const size_t nwaves = (size_t)std::max(sim_grid, 1) * kWaves;
  ZPL_TRY(ensure(c, c->list_v, sizeof(int64_t) * nwaves * kListCap));
  ZPL_TRY(ensure(c, c->list_c, sizeof(uint32_t) * nwaves * kListCap));
  ZPL_TRY(ensure(c, c->wslots, (size_t)kWaveSlotBytes * 64 * nwaves));
  L.hstride = heavy_stride(P.max_n);
  int hg = (int)std::min<int64_t>((int64_t)P.hunits.size() + 64, (int64_t)c->n_cu * 2);
  // keep the heavy scratch (one area per wave) within a quarter of the budget
  while (hg > 1 && (uint64_t)hg * kHeavyWaves * L.hstride * 8 > c->budget / 4) hg /= 2;
  L.heavy_grid = hg;
  ZPL_TRY(ensure(c, c->heavy, sizeof(int64_t) * (size_t)hg * kHeavyWaves * L.hstride));
  if (need_dbuf) ZPL_TRY(ensure(c, c->dbuf, sizeof(double) * (size_t)P.total_R));
  // bracket gather: at most ~12% of a cell's replicates fall in a bracket
  int64_t maxR = 1;
  for (const DevCell& d : P.cells) maxR = std::max(maxR, d.R);
  L.gcap = std::min<int64_t>(kSelGather, maxR * 3 / 20 + 1024);
  L.maxR = maxR;
  // gather areas, then 32 bytes of selection state per (cell, quantile)
  if (n_q > 0)
    ZPL_TRY(ensure(c, c->gather, sizeof(uint64_t) * (size_t)nc * kSelQ * L.gcap +
                                     (size_t)32 * nc * kSelQ));
  return ZPL_OK;
}

// Enqueue everything after the plan upload: counters, tables, simulation,
// heavy pass, selection.  Kernel launches only (graph-capturable).
zpl_status enqueue_run(zpl_ctx* c, const Plan& P, int launch, const Launch& L, Outputs out,
                       const double* Dsel, int n_q, hipStream_t s, bool timed) {
  const int nc = (int)P.cells.size();
  auto mark = [&](int k) -> hipError_t {
    return timed ? hipEventRecord(c->ev[k], s) : hipSuccess;
  };
  char* plan = (char*)c->plan.p;
  char* ctr = (char*)c->ctr.p;
  DevCell* dcells = (DevCell*)plan;
  uint32_t* queues = (uint32_t*)ctr;
  uint32_t* escc = (uint32_t*)(ctr + L.lay.esc);
  uint32_t* err = (uint32_t*)(ctr + L.lay.err);
  bool any_trunc = false;
  for (const DevCell& d : P.cells) any_trunc = any_trunc || d.K != 0u;
  HIP_TRY(mark(0));
  // the table kernel also clears the counters
  HIP_TRY(launch_tables(dcells, nc, (double*)c->tables.p, (uint16_t*)c->guides.p, c->ln, s,
                        any_trunc, queues, L.lay.ctr_words));
  HIP_TRY(mark(1));
  const Unit* units = (const Unit*)(plan + L.lay.units);
  if (launch == ZPL_LAUNCH_PLAIN) {
    for (int i = 0; i < nc; ++i) {
      const int b = P.cell_unit_begin[i], e = P.cell_unit_end[i];
      if (e <= b) continue;
      const int grid = std::min(e - b, c->n_cu);
      HIP_TRY(launch_simulate(grid, dcells, (const double*)c->tables.p,
                              (const uint16_t*)c->guides.p, c->ln, units + b, e - b,
                              queues + 8 + i, out, (uint64_t*)c->esc.p, escc, c->esc_cap,
                              (int64_t*)c->list_v.p, (uint32_t*)c->list_c.p, c->wslots.p,
                              err, s));
    }
  } else {
    HIP_TRY(launch_simulate(L.sim_grid, dcells, (const double*)c->tables.p,
                            (const uint16_t*)c->guides.p, c->ln, units, (int)P.units.size(),
                            queues + 0, out, (uint64_t*)c->esc.p, escc, c->esc_cap,
                            (int64_t*)c->list_v.p, (uint32_t*)c->list_c.p, c->wslots.p,
                            err, s));
  }
  HIP_TRY(mark(2));
  HIP_TRY(launch_heavy(L.heavy_grid, dcells, (const double*)c->tables.p,
                       (const uint16_t*)c->guides.p, c->ln, (const Unit*)(plan + L.lay.hunits),
                       (int)P.hunits.size(), (const uint64_t*)c->esc.p, escc, c->esc_cap,
                       queues + 2, out, (int64_t*)c->heavy.p, L.hstride, s));
  HIP_TRY(mark(3));
  if (n_q > 0 && Dsel)
    HIP_TRY(launch_select(Dsel, dcells, nc, n_q, (const uint32_t*)(plan + L.lay.qnum),
                          (const uint32_t*)(plan + L.lay.qden), (double*)(ctr + L.lay.qout),
                          (uint64_t*)c->gather.p, L.gcap, L.maxR, c->n_cu, s));
  HIP_TRY(mark(4));
  return ZPL_OK;
}

zpl_status err_word_status(uint32_t e) {
  if (e & kErrEscOverflow)
    return fail(ZPL_ENOMEM, "escalation list overflow (too many replicates exceeded their form's capacity)");
  return ZPL_OK;
}

zpl_status check_err_word(zpl_ctx* c, hipStream_t s) {
  uint32_t e = 0;
  HIP_TRY(hipMemcpyAsync(&e, (char*)c->ctr.p + c->err_off, sizeof e, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return err_word_status(e);
}

// Simulation of a plan with outputs; shared by zpl_simulate_cells and the
// bootstrap.  quantiles may be NULL.
zpl_status run_cells(zpl_ctx* c, const zpl_cell* cells, int n_cells, const uint32_t* q_num,
                     const uint32_t* q_den, int n_q, double* quantiles, Outputs out,
                     const zpl_sim_opts* opts, hipStream_t s, const int64_t* rlo = nullptr) {
  zpl_sim_opts o = {ZPL_LAUNCH_BATCHED, ZPL_FORM_AUTO, 0, 0};
  if (opts) o = *opts;
  if (o.launch != ZPL_LAUNCH_BATCHED && o.launch != ZPL_LAUNCH_PLAIN)
    return fail(ZPL_EINVAL, "opts.launch must be ZPL_LAUNCH_BATCHED or ZPL_LAUNCH_PLAIN");
  if (o.form < ZPL_FORM_AUTO || o.form > ZPL_FORM_HEAVY)
    return fail(ZPL_EINVAL, "opts.form out of range");
  if (o.reserved != 0) return fail(ZPL_EINVAL, "opts.reserved must be 0");
  if (n_q < 0 || (n_q > 0 && (!q_num || !q_den)))
    return fail(ZPL_EINVAL, "quantile arrays missing");
  for (int i = 0; i < n_q; ++i)
    if (q_den[i] == 0 || q_num[i] >= q_den[i])
      return fail(ZPL_EINVAL, "quantile %d: need num < den (got %u/%u)", i, q_num[i], q_den[i]);
  if (rlo && (o.use_graph || n_q > 0))
    return fail(ZPL_EINVAL, "replicate windows run without graphs or quantiles");
  Plan P;
  ZPL_TRY(make_plan(cells, n_cells, o.form, P, &c->tune, c->n_cu, rlo));
  if (o.launch == ZPL_LAUNCH_PLAIN) plain_unit_order(P);
  const bool need_sel = quantiles && n_q > 0;
  const bool need_dbuf = need_sel && out.D == nullptr;
  Launch L;
  ZPL_TRY(prepare(c, P, n_q, need_dbuf, L));
  if (need_dbuf) out.D = (double*)c->dbuf.p;
  // graph key: everything the captured launches depend on
  const bool graphed = o.use_graph && o.launch == ZPL_LAUNCH_BATCHED;
  std::vector<char> key;
  auto put = [&](const void* p, size_t b) {
    if (!graphed) return;
    const char* q = (const char*)p;
    key.insert(key.end(), q, q + b);
  };
  put(&o, sizeof o);
  put(&n_cells, sizeof n_cells);
  put(cells, sizeof(zpl_cell) * (size_t)n_cells);
  put(&n_q, sizeof n_q);
  if (n_q) {
    put(q_num, sizeof(uint32_t) * n_q);
    put(q_den, sizeof(uint32_t) * n_q);
  }
  put(&out, sizeof out);
  put(&s, sizeof s);
  // the plan itself: it also depends on the tuning table and the device
  put(P.cells.data(), sizeof(DevCell) * P.cells.size());
  put(P.units.data(), sizeof(Unit) * P.units.size());
  put(P.hunits.data(), sizeof(Unit) * P.hunits.size());
  const bool replay = o.use_graph && o.launch == ZPL_LAUNCH_BATCHED && c->graph_valid &&
                      c->graph_key == key;
  // pinned staging: the plan upload, then (from dl_off) the error word and
  // the quantiles on their way back
  const PlanLayout& Y = L.lay;
  const size_t dl_off = (Y.plan_bytes + 255) & ~(size_t)255;
  const size_t dl_bytes = need_sel ? Y.ctr_bytes - Y.err : 0;
  ZPL_TRY(ensure_pinned(c, dl_off + dl_bytes));
  char* pin = (char*)c->pin;
  if (!replay || c->plan_gen != c->graph_plan_gen) {
    HIP_TRY(hipStreamSynchronize(s));  // the staging area may still be in use
    std::memcpy(pin, P.cells.data(), sizeof(DevCell) * P.cells.size());
    std::memcpy(pin + Y.units, P.units.data(), sizeof(Unit) * P.units.size());
    std::memcpy(pin + Y.hunits, P.hunits.data(), sizeof(Unit) * P.hunits.size());
    if (n_q) {
      std::memcpy(pin + Y.qnum, q_num, sizeof(uint32_t) * n_q);
      std::memcpy(pin + Y.qden, q_den, sizeof(uint32_t) * n_q);
    }
    HIP_TRY(hipMemcpyAsync(c->plan.p, pin, Y.plan_bytes, hipMemcpyHostToDevice, s));
    ++c->plan_gen;
  }
  const double* Dsel = need_sel ? out.D : nullptr;
  if (o.use_graph && o.launch == ZPL_LAUNCH_BATCHED) {
    if (!replay) {
      if (c->graph_valid) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_valid = false;
      }
      // the plan upload above must be complete before a replay on any stream
      HIP_TRY(hipStreamSynchronize(s));
      if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      hipGraph_t g;
      HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      zpl_status st =
          enqueue_run(c, P, o.launch, L, out, Dsel, need_sel ? n_q : 0, c->cap_stream, false);
      hipError_t ce = hipStreamEndCapture(c->cap_stream, &g);
      if (st != ZPL_OK) {
        if (ce == hipSuccess) (void)hipGraphDestroy(g);
        return st;
      }
      HIP_TRY(ce);
      hipError_t ie = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_TRY(ie);
      c->graph_valid = true;
      c->graph_key = key;
    }
    c->graph_plan_gen = c->plan_gen;
    HIP_TRY(hipGraphLaunch(c->graph_exec, s));
    c->timed = false;
  } else {
    if (c->timing && !c->ev[0])
      for (hipEvent_t& e : c->ev) HIP_TRY(hipEventCreate(&e));
    ZPL_TRY(enqueue_run(c, P, o.launch, L, out, Dsel, need_sel ? n_q : 0, s, c->timing));
    c->timed = c->timing;
  }
  if (need_sel) {
    // error word and quantiles in one copy to pinned memory
    HIP_TRY(hipMemcpyAsync(pin + dl_off, (char*)c->ctr.p + Y.err, dl_bytes, hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    uint32_t e;
    std::memcpy(&e, pin + dl_off, sizeof e);
    ZPL_TRY(err_word_status(e));
    std::memcpy(quantiles, pin + dl_off + (Y.qout - Y.err), sizeof(double) * (size_t)n_cells * n_q);
  }
  return ZPL_OK;
}

// Measures the cost of each eligible form at every grid point: a probe cell
// with enough replicates to give every compute unit one unit of work (lane
// and wave forms: kBlock replicates per workgroup; heavy form: 8 per
// workgroup of its grid), timed with events around the simulation and heavy
// launches (table build excluded), best of two runs.
zpl_status autotune_grid(zpl_ctx* c, const double* alphas, int na, const int64_t* ns, int nn,
                         std::vector<zpl_tune_entry>& out, hipStream_t s) {
  out.assign((size_t)na * nn, zpl_tune_entry{});
  const bool was_timing = c->timing;
  if (!c->ev[0])
    for (hipEvent_t& e : c->ev) HIP_TRY(hipEventCreate(&e));
  c->timing = true;
  zpl_status st = ZPL_OK;
  for (int ia = 0; ia < na && st == ZPL_OK; ++ia)
    for (int in = 0; in < nn && st == ZPL_OK; ++in) {
      zpl_tune_entry& e = out[(size_t)ia * nn + in];
      e.alpha = alphas[ia];
      e.n = ns[in];
      for (int f = 0; f < 3 && st == ZPL_OK; ++f) {
        e.ns_per_replicate[f] = -1.0;
        if (!form_eligible((uint32_t)f, alphas[ia], ns[in])) continue;
        const int64_t R = f == kModeHeavy ? (int64_t)c->n_cu * 2 * 8 : (int64_t)c->n_cu * kBlock;
        st = ensure(c, c->dbuf, sizeof(double) * (size_t)R);
        if (st != ZPL_OK) break;
        const zpl_cell z = {alphas[ia], ns[in], R, 0x7475656eull, (uint32_t)(ia * nn + in), 0};
        const zpl_sim_opts o = {ZPL_LAUNCH_BATCHED, f + 1, 0, 0};
        Outputs po{(double*)c->dbuf.p, nullptr, nullptr, nullptr, nullptr};
        double best = -1.0;
        for (int rep = 0; rep < 2 && st == ZPL_OK; ++rep) {
          st = run_cells(c, &z, 1, nullptr, nullptr, 0, nullptr, po, &o, s);
          if (st != ZPL_OK) break;
          if (hipEventSynchronize(c->ev[3]) != hipSuccess) {
            st = fail(ZPL_EDEVICE, "autotune: event wait failed");
            break;
          }
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, c->ev[1], c->ev[3]) != hipSuccess) {
            st = fail(ZPL_EDEVICE, "autotune: event timing failed");
            break;
          }
          const double v = (double)ms * 1e6 / (double)R;
          if (best < 0.0 || v < best) best = v;
        }
        if (st == ZPL_OK) st = check_err_word(c, s);
        e.ns_per_replicate[f] = best;
      }
    }
  c->timing = was_timing;
  c->timed = false;
  return st;
}

zpl_status fit_device(zpl_ctx* c, const int64_t* xd, int64_t n, hipStream_t s, double* ahat,
                      double* D, uint32_t* flags, uint32_t* status, uint32_t K = 0) {
  const int64_t stride = heavy_stride(n);
  ZPL_TRY(ensure(c, c->fit_ptrs, sizeof(int64_t*)));
  ZPL_TRY(ensure(c, c->fit_ns, sizeof(int64_t)));
  ZPL_TRY(ensure(c, c->fit_out, sizeof(double) * 2 + sizeof(uint32_t) * 2));
  ZPL_TRY(ensure(c, c->fit_st, sizeof(uint32_t) * 2));
  ZPL_TRY(ensure(c, c->heavy, grow_size(sizeof(int64_t) * (size_t)stride)));
  ZPL_TRY(ensure_pinned(c, 64));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t* pin = (int64_t*)c->pin;
  pin[0] = (int64_t)(intptr_t)xd;
  pin[1] = n;
  HIP_TRY(hipMemcpyAsync(c->fit_ptrs.p, &pin[0], sizeof(int64_t), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->fit_ns.p, &pin[1], sizeof(int64_t), hipMemcpyHostToDevice, s));
  double* o = (double*)c->fit_out.p;
  uint32_t* of = (uint32_t*)(o + 2);
  // a large dataset is read, histogrammed and sorted by a whole workgroup
  // (the same list and finish, so the same bits as the one-wave kernel)
  if (n >= kFitBlockMin)
    HIP_TRY(launch_fit_block(xd, n, c->ln, (int64_t*)c->heavy.p, stride, o, o + 1, of,
                             (uint32_t*)c->fit_st.p, K, s));
  else
    HIP_TRY(launch_fit(1, (const int64_t* const*)c->fit_ptrs.p, (const int64_t*)c->fit_ns.p, 1,
                       c->ln, (int64_t*)c->heavy.p, stride, o, o + 1, of,
                       (uint32_t*)c->fit_st.p, K, s));
  char* hp = (char*)c->pin + 16;
  HIP_TRY(hipMemcpyAsync(hp, o, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hp + 16, of, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hp + 20, c->fit_st.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(ahat, hp, sizeof(double));
  std::memcpy(D, hp + 8, sizeof(double));
  std::memcpy(flags, hp + 16, sizeof(uint32_t));
  std::memcpy(status, hp + 20, sizeof(uint32_t));
  return ZPL_OK;
}

zpl_status stage_x(zpl_ctx* c, const int64_t* x, int64_t n, int32_t on_dev, hipStream_t s,
                   const int64_t** xd) {
  if (on_dev) {
    *xd = x;
    return ZPL_OK;
  }
  const size_t bytes = sizeof(int64_t) * (size_t)n;
  ZPL_TRY(ensure(c, c->fit_x, bytes <= kPinStageMax ? grow_size(bytes) : bytes));
  if (bytes <= kPinStageMax) {
    // a pageable source is copied by the runtime in small staged pieces;
    // one host copy into pinned memory and one DMA are several times faster
    if (c->pin_x_bytes < bytes) {
      const size_t want = grow_size(bytes);
      HIP_TRY(hipStreamSynchronize(s));
      if (c->pin_x) HIP_TRY(hipHostFree(c->pin_x));
      c->pin_x = nullptr;
      c->pin_x_bytes = 0;
      HIP_TRY(hipHostMalloc(&c->pin_x, want, hipHostMallocDefault));
      c->pin_x_bytes = want;
    }
    HIP_TRY(hipStreamSynchronize(s));  // the previous staged copy has finished
    std::memcpy(c->pin_x, x, bytes);
    HIP_TRY(hipMemcpyAsync(c->fit_x.p, c->pin_x, bytes, hipMemcpyHostToDevice, s));
  } else {
    HIP_TRY(hipMemcpyAsync(c->fit_x.p, x, bytes, hipMemcpyHostToDevice, s));
  }
  *xd = (const int64_t*)c->fit_x.p;
  return ZPL_OK;
}

}  // namespace


// ===========================================================================
// Serving: continuous batching of bootstrap p-value requests.
//
// A scheduler thread owns an internal context and stream.  Each iteration:
//   1. admits queued requests, oldest first, while an active slot is free and
//      their device memory fits the budget (the fit's dataset and scratch
//      while it runs, and 8 bytes per bootstrap replicate until the request
//      completes);
//   2. fits the newly admitted datasets (eq. 2 and eq. 3) in one batched
//      launch (one wavefront per dataset below 2,048 values, one workgroup per
//      larger dataset);
//   3. runs one window of replicates of every active request's bootstrap, all
//      of them as the cells of one batched simulation, the windows sized so
//      that the launch holds about one time slice of work shared equally
//      between the requests (a request needing less than its share finishes
//      in this launch and its share goes to the others);
//   4. counts D_b >= D_obs in each window and completes every request whose
//      last window ran.
// A request that arrives while a launch runs joins the next one and shares
// the device with the requests already in flight, so a short request is not
// held behind a long bootstrap.  Every draw is a pure function of (seed,
// stream, replicate) and each replicate runs exactly once, so a request's
// result does not depend on what it shares the launches with.
// ===========================================================================
namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  std::vector<int64_t> x;    // host dataset (submitted from host memory)
  int64_t* xdev = nullptr;   // device copy (submitted from device memory), stream-ordered
  int64_t n = 0;
  int64_t B = 0;
  uint64_t seed = 0;
  uint32_t stream_id = 0;
  Clock::time_point t_submit, t_start, t_done;
  bool done = false;
  zpl_status status = ZPL_OK;
  double ahat = 0.0, D = 0.0, p = 0.0;
  uint32_t flags = 0;
  // scheduling state (scheduler thread only)
  int64_t next = 0;          // first bootstrap replicate not yet run
  uint64_t ge = 0;           // replicates so far with D_b >= D_obs
  double cost = 0.0;         // estimated ns per replicate, device busy
  size_t held = 0;           // bytes charged while active
  int32_t mix = 0;           // most requests that shared a launch with it
  int32_t launches = 0;      // simulation launches that ran its replicates
};

// Device memory a request holds while active: the D values of its
// replicates in the slice buffer (at most all B of them in one launch).
size_t held_bytes(const Req& r) { return (size_t)r.B * 8 + 4096; }

// Transient device memory of fitting a set of datasets: the concatenated
// data, the per-set descriptors and outputs, the one-wave fits' scratch
// (one area per wavefront of the batched launch, each sized for the largest
// small dataset) and one workgroup fit's scratch, reused by every large one.
size_t fit_bytes(int64_t total_n, int n_sets, int64_t max_small, int n_small, int64_t max_large,
                 int n_cu) {
  size_t b = (size_t)total_n * 8 + (size_t)n_sets * 64 + 4096;
  if (n_small > 0)
    b += (size_t)std::min(n_small, 2 * n_cu) * (size_t)heavy_stride(max_small) * 8;
  if (max_large > 0) b += (size_t)heavy_stride(max_large) * 8;
  return b;
}

// Estimated cost of one bootstrap replicate (ns with the device busy): the
// tuned cost of the cheapest eligible form when a table is installed, else
// about 2.2 ps per draw, more with heavy tails, and 2.5 ns per replicate (a
// fit to MI355X's tuned costs over the table's exponents and sizes).
double replicate_cost(const zpl_ctx* c, double alpha, int64_t n) {
  double v;
  (void)choose_form(alpha, n, &c->tune, 0, 1, c->n_cu, -1.0, &v);
  if (v > 0.0) return v;
  return 2.2e-3 * (double)n * (1.0 + 90.0 * tail_prob(alpha, kHW)) + 2.5;
}

}  // namespace

struct Server {
  zpl_ctx* eng = nullptr;  // internal context used only by the scheduler thread
  hipStream_t stream = nullptr;
  hipStream_t submit_stream = nullptr;  // device datasets are copied on it
  uint64_t budget = 8ull << 30;
  int max_active = 256;
  int max_queue = 1 << 16;
  double slice_ns = 4e6;   // target work per simulation launch
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string fatal;  // scheduler error, reported by later calls
  uint64_t iterations = 0, served = 0;
  size_t used = 0;    // bytes held by active requests (scheduler thread)
  std::vector<Req*> active;

  void loop();
  zpl_status fit_fresh(std::vector<Req*>& fresh);
  zpl_status run_slice(std::vector<Req*>& finished);
  void complete(Req* r, zpl_status st);
};

// Publishes a result (caller holds no lock).
void Server::complete(Req* r, zpl_status st) {
  std::lock_guard<std::mutex> lk(mu);
  r->status = st;
  r->t_done = Clock::now();
  r->done = true;
  if (r->xdev) {
    (void)hipFreeAsync(r->xdev, stream);
    r->xdev = nullptr;
  }
  r->x.clear();
  r->x.shrink_to_fit();
  ++served;
  cv.notify_all();
}

// Uploads and fits the newly admitted datasets; a request that fails here
// (invalid values, no root) is completed at once, the others become active.
zpl_status Server::fit_fresh(std::vector<Req*>& fresh) {
  zpl_ctx* c = eng;
  hipStream_t s = stream;
  const int nb = (int)fresh.size();
  int64_t total = 0;
  for (Req* r : fresh) total += r->n;
  // 1. datasets -> one device buffer (host data through pinned staging)
  const size_t pin_need = sizeof(int64_t) * (size_t)total + (sizeof(int64_t) * 2 + 64) * nb + 4096;
  ZPL_TRY(ensure_pinned(c, pin_need));
  HIP_TRY(hipStreamSynchronize(s));
  char* pin = (char*)c->pin;
  int64_t* px = (int64_t*)pin;
  ZPL_TRY(ensure(c, c->fit_x, sizeof(int64_t) * (size_t)std::max<int64_t>(total, 1)));
  int64_t* fx = (int64_t*)c->fit_x.p;
  int64_t off = 0;
  for (Req* r : fresh) {
    if (r->xdev)
      HIP_TRY(hipMemcpyAsync(fx + off, r->xdev, sizeof(int64_t) * (size_t)r->n,
                             hipMemcpyDeviceToDevice, s));
    else
      std::memcpy(px + off, r->x.data(), sizeof(int64_t) * (size_t)r->n);
    off += r->n;
  }
  // host-submitted data: one copy of the staged runs (device runs are skipped)
  off = 0;
  for (int i = 0; i < nb;) {
    if (fresh[i]->xdev) {
      off += fresh[i]->n;
      ++i;
      continue;
    }
    int64_t run = 0;
    const int64_t start = off;
    while (i < nb && !fresh[i]->xdev) {
      run += fresh[i]->n;
      off += fresh[i]->n;
      ++i;
    }
    HIP_TRY(hipMemcpyAsync(fx + start, px + start, sizeof(int64_t) * (size_t)run,
                           hipMemcpyHostToDevice, s));
  }
  // 2. fits: small datasets one wavefront each in one launch, large ones a
  //    workgroup each (the same bits as zpl_fit either way)
  std::vector<int> small, large;
  int64_t max_small = 1, max_large = 0;
  for (int i = 0; i < nb; ++i) {
    if (fresh[i]->n >= kFitBlockMin) {
      large.push_back(i);
      max_large = std::max(max_large, fresh[i]->n);
    } else {
      small.push_back(i);
      max_small = std::max(max_small, fresh[i]->n);
    }
  }
  int64_t* pptr = (int64_t*)(pin + sizeof(int64_t) * total);
  int64_t* pns = pptr + nb;
  std::vector<int64_t> xoff(nb);
  off = 0;
  for (int i = 0; i < nb; ++i) {
    xoff[i] = off;
    off += fresh[i]->n;
  }
  for (size_t k = 0; k < small.size(); ++k) {
    pptr[k] = (int64_t)(intptr_t)(fx + xoff[small[k]]);
    pns[k] = fresh[small[k]]->n;
  }
  ZPL_TRY(ensure(c, c->fit_ptrs, sizeof(int64_t) * nb));
  ZPL_TRY(ensure(c, c->fit_ns, sizeof(int64_t) * nb));
  ZPL_TRY(ensure(c, c->fit_out, (sizeof(double) * 2 + sizeof(uint32_t) * 2) * nb));
  ZPL_TRY(ensure(c, c->fit_st, sizeof(uint32_t) * nb));
  double* fa = (double*)c->fit_out.p;
  double* fd = fa + nb;
  uint32_t* ff = (uint32_t*)(fd + nb);
  uint32_t* fs = (uint32_t*)c->fit_st.p;
  const int ns_small = (int)small.size();
  const int grid = std::min(ns_small, c->n_cu * 2);
  const int64_t sstride = heavy_stride(max_small);
  const int64_t lstride = max_large > 0 ? heavy_stride(max_large) : 0;
  ZPL_TRY(ensure(c, c->heavy, sizeof(int64_t) * (size_t)std::max<int64_t>(
                                  (int64_t)grid * sstride, std::max<int64_t>(lstride, 1))));
  if (ns_small > 0) {
    HIP_TRY(hipMemcpyAsync(c->fit_ptrs.p, pptr, sizeof(int64_t) * ns_small,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->fit_ns.p, pns, sizeof(int64_t) * ns_small, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fit(grid, (const int64_t* const*)c->fit_ptrs.p, (const int64_t*)c->fit_ns.p,
                       ns_small, c->ln, (int64_t*)c->heavy.p, sstride, fa, fd, ff, fs, 0u, s));
  }
  // large ones after the small ones' outputs, sharing one scratch area
  for (size_t k = 0; k < large.size(); ++k) {
    const int o = ns_small + (int)k;
    const int i = large[k];
    HIP_TRY(launch_fit_block(fx + xoff[i], fresh[i]->n, c->ln, (int64_t*)c->heavy.p,
                             heavy_stride(fresh[i]->n), fa + o, fd + o, ff + o, fs + o, 0u, s));
  }
  double* ha = (double*)(pns + nb);
  double* hd = ha + nb;
  uint32_t* hf = (uint32_t*)(hd + nb);
  uint32_t* hs = hf + nb;
  HIP_TRY(hipMemcpyAsync(ha, fa, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hd, fd, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hf, ff, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hs, fs, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // outputs are in small-then-large order
  std::vector<int> order(small);
  order.insert(order.end(), large.begin(), large.end());
  for (int o = 0; o < nb; ++o) {
    Req* r = fresh[order[o]];
    r->ahat = ha[o];
    r->D = hd[o];
    r->flags = hf[o];
    if (r->xdev) {
      (void)hipFreeAsync(r->xdev, s);
      r->xdev = nullptr;
    }
    r->x.clear();
    r->x.shrink_to_fit();
    if (hs[o] != 0u) {
      used -= r->held;
      complete(r, ZPL_EINVAL);
      continue;
    }
    if (!(r->ahat >= kMinAlpha)) {
      used -= r->held;
      complete(r, ZPL_ENOCONV);
      continue;
    }
    r->cost = replicate_cost(c, r->ahat, r->n);
    active.push_back(r);
  }
  return ZPL_OK;
}

// One simulation launch over a window of every active request's bootstrap,
// then the counts; requests whose last window ran go to `finished`.
zpl_status Server::run_slice(std::vector<Req*>& finished) {
  zpl_ctx* c = eng;
  hipStream_t s = stream;
  const int na = (int)active.size();
  // windows: the slice's work shared equally, smallest remaining first (a
  // request needing less than its share leaves the rest to the others)
  std::vector<int> ord(na);
  for (int i = 0; i < na; ++i) ord[i] = i;
  auto rem_work = [&](int i) { return (double)(active[i]->B - active[i]->next) * active[i]->cost; };
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return rem_work(a) < rem_work(b); });
  std::vector<int64_t> win(na, 0);
  double budget = slice_ns;
  for (int k = 0; k < na; ++k) {
    const int i = ord[k];
    Req* r = active[i];
    const double share = budget / (double)(na - k);
    const double take = std::min(rem_work(i), share);
    budget -= take;
    int64_t w = (int64_t)std::ceil(take / std::max(r->cost, 1e-9));
    w = std::max<int64_t>(1, std::min<int64_t>(w, r->B - r->next));
    win[i] = w;
  }
  std::vector<zpl_cell> cells(na);
  std::vector<int64_t> rlo(na), base(na);
  int64_t total = 0;
  for (int i = 0; i < na; ++i) {
    Req* r = active[i];
    cells[i] = zpl_cell{r->ahat, r->n, win[i], r->seed, r->stream_id, 0, 0};
    rlo[i] = r->next;
    base[i] = total;
    total += win[i];
  }
  ZPL_TRY(ensure(c, c->boot_d, sizeof(double) * (size_t)total));
  Outputs out{(double*)c->boot_d.p, nullptr, nullptr, nullptr, nullptr};
  ZPL_TRY(run_cells(c, cells.data(), na, nullptr, nullptr, 0, nullptr, out, nullptr, s,
                    rlo.data()));
  // counts of D_b >= D_obs per window: cells {out_off = window start, R = window}
  ZPL_TRY(ensure(c, c->count, (sizeof(unsigned long long) + sizeof(double)) * na +
                                  sizeof(DevCell) * na + 64));
  unsigned long long* cnt = (unsigned long long*)c->count.p;
  double* ddev = (double*)(cnt + na);
  DevCell* ccells = (DevCell*)(ddev + na);
  HIP_TRY(hipStreamSynchronize(s));  // the plan upload used the staging area
  ZPL_TRY(ensure_pinned(c, (sizeof(double) + sizeof(unsigned long long)) * na +
                               sizeof(DevCell) * na + 64));
  double* pd = (double*)c->pin;
  DevCell* pc = (DevCell*)(pd + na);
  unsigned long long* hc = (unsigned long long*)(pc + na);
  int64_t maxw = 1;
  for (int i = 0; i < na; ++i) {
    pd[i] = active[i]->D;
    std::memset(&pc[i], 0, sizeof(DevCell));
    pc[i].out_off = base[i];
    pc[i].R = win[i];
    maxw = std::max(maxw, win[i]);
  }
  HIP_TRY(hipMemcpyAsync(ddev, pd, sizeof(double) * na, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ccells, pc, sizeof(DevCell) * na, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_fill_u32((uint32_t*)cnt, 2 * na, 0u, s));
  HIP_TRY(launch_count_cells((const double*)c->boot_d.p, ccells, na, ddev, cnt, maxw, s));
  HIP_TRY(hipMemcpyAsync(hc, cnt, sizeof(unsigned long long) * na, hipMemcpyDeviceToHost, s));
  ZPL_TRY(check_err_word(c, s));  // synchronises the stream
  std::vector<Req*> still;
  for (int i = 0; i < na; ++i) {
    Req* r = active[i];
    r->ge += hc[i];
    r->next += win[i];
    r->launches += 1;
    r->mix = std::max(r->mix, na);
    if (r->next >= r->B)
      finished.push_back(r);
    else
      still.push_back(r);
  }
  active.swap(still);
  return ZPL_OK;
}

void Server::loop() {
  if (hipSetDevice(eng->device) != hipSuccess ||
      hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    fatal = "serving: could not create the scheduler stream";
    stop = true;
  }
  for (;;) {
    std::vector<Req*> fresh;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (active.empty()) cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty() && active.empty() && stop) break;
      if (!fatal.empty()) {
        // no device work after a fatal error: fail everything still here
        std::vector<Req*> all(queue.begin(), queue.end());
        all.insert(all.end(), active.begin(), active.end());
        queue.clear();
        active.clear();
        for (Req* r : all) {
          r->status = ZPL_EDEVICE;
          r->t_done = Clock::now();
          r->done = true;
        }
        cv.notify_all();
        if (stop) break;
        continue;
      }
      // admission: oldest first, while a slot is free and the memory the
      // request holds plus the admitted fits' transient memory fit
      int64_t tot = 0, ms = 1, ml = 0;
      int nsml = 0;
      while (!queue.empty() && (int)(active.size() + fresh.size()) < max_active) {
        Req* r = queue.front();
        const int64_t t2 = tot + r->n;
        const bool lg = r->n >= kFitBlockMin;
        const int64_t ms2 = lg ? ms : std::max(ms, r->n), ml2 = lg ? std::max(ml, r->n) : ml;
        const int ns2 = nsml + (lg ? 0 : 1);
        const size_t h = held_bytes(*r);
        const size_t need = used + h +
                            fit_bytes(t2, (int)fresh.size() + 1, ms2, ns2, ml2, eng->n_cu);
        const size_t alone = h + fit_bytes(r->n, 1, lg ? 1 : r->n, lg ? 0 : 1, lg ? r->n : 0,
                                           eng->n_cu);
        if (alone > budget) {  // can never be admitted
          queue.pop_front();
          r->status = ZPL_ENOMEM;
          r->t_done = Clock::now();
          r->done = true;
          if (r->xdev) {
            (void)hipFreeAsync(r->xdev, stream);
            r->xdev = nullptr;
          }
          cv.notify_all();
          continue;
        }
        if (need > budget) break;  // admitted when memory frees up
        queue.pop_front();
        r->held = h;
        used += h;
        r->t_start = Clock::now();
        fresh.push_back(r);
        tot = t2;
        ms = ms2;
        ml = ml2;
        nsml = ns2;
      }
    }
    zpl_status st = ZPL_OK;
    if (!fresh.empty()) {
      st = fit_fresh(fresh);
      if (st == ZPL_ENOMEM) {  // only these requests fail
        for (Req* r : fresh)
          if (!r->done && std::find(active.begin(), active.end(), r) == active.end()) {
            used -= r->held;
            complete(r, ZPL_ENOMEM);
          }
        st = ZPL_OK;
      }
    }
    std::vector<Req*> finished;
    if (st == ZPL_OK && !active.empty()) {
      st = run_slice(finished);
      if (st == ZPL_ENOMEM) {  // the launch did not fit: fail the active requests only
        std::vector<Req*> failed;
        failed.swap(active);
        for (Req* r : failed) {
          used -= r->held;
          complete(r, ZPL_ENOMEM);
        }
        st = ZPL_OK;
      }
    }
    for (Req* r : finished) {
      used -= r->held;
      r->p = (double)r->ge / (double)r->B;
      complete(r, ZPL_OK);
    }
    if (st != ZPL_OK) {
      std::lock_guard<std::mutex> lk(mu);
      fatal = "serving: " + g_err;
      cv.notify_all();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      ++iterations;
    }
  }
  if (stream) {
    (void)hipStreamSynchronize(stream);
    (void)hipStreamDestroy(stream);
  }
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* zpl_last_error(void) { return g_err.c_str(); }

zpl_status zpl_create(zpl_ctx** out, int32_t device, uint64_t mem_budget_bytes) {
  g_err.clear();
  if (!out) return fail(ZPL_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev)
    return fail(ZPL_EINVAL, "device %d out of range (%d devices)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  zpl_ctx* c = new zpl_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->budget = mem_budget_bytes ? mem_budget_bytes : (64ull << 30);
  hipError_t e = hipMalloc(&c->ln, sizeof(double) * (kH + 2));
  if (e != hipSuccess) {
    delete c;
    return fail(ZPL_ENOMEM, "hipMalloc(ln): %s", hipGetErrorString(e));
  }
  // the allocation-free fit's array: its device address on this GPU (the
  // symbol itself is only a host-side stand-in)
  e = noalloc_scratch_address(&c->noalloc_scratch);
  if (e != hipSuccess || !c->noalloc_scratch) {
    (void)hipFree(c->ln);
    delete c;
    return fail(ZPL_EDEVICE, "hipGetSymbolAddress(noalloc scratch): %s", hipGetErrorString(e));
  }
  e = launch_ln_table(c->ln, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(c->ln);
    delete c;
    return fail(ZPL_EDEVICE, "ln table: %s", hipGetErrorString(e));
  }
  *out = c;
  return ZPL_OK;
}

void zpl_destroy(zpl_ctx* c) {
  if (!c) return;
  if (c->server) (void)zpl_serve_stop(c);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->graph_valid) (void)hipGraphExecDestroy(c->graph_exec);
  DevBuf* bufs[] = {&c->plan,   &c->ctr,      &c->tables, &c->guides, &c->esc,
                    &c->list_v, &c->list_c,   &c->wslots, &c->heavy,  &c->gather,
                    &c->dbuf,   &c->fit_x,    &c->fit_ptrs, &c->fit_ns, &c->fit_out,
                    &c->fit_st, &c->count,    &c->boot_d, &c->scan};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (c->ln) (void)hipFree(c->ln);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->pin_x) (void)hipHostFree(c->pin_x);
  delete c;
}

zpl_status zpl_simulate_cells(zpl_ctx* c, const zpl_cell* cells, int32_t n_cells,
                              const uint32_t* q_num, const uint32_t* q_den, int32_t n_q,
                              double* quantiles, double* d_out, double* alpha_hat_out,
                              uint32_t* flags_out, uint64_t* fingerprint_out,
                              const zpl_sim_opts* opts, void* stream) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  if (n_cells < 1 || !cells) return fail(ZPL_EINVAL, "need at least one cell");
  HIP_TRY(hipSetDevice(c->device));
  Outputs out{d_out, alpha_hat_out, flags_out, fingerprint_out, nullptr};
  return run_cells(c, cells, n_cells, q_num, q_den, quantiles ? n_q : 0, quantiles, out, opts,
                   (hipStream_t)stream);
}

zpl_status zpl_critical_table(zpl_ctx* c, const double* gammas, int32_t n_gamma,
                              const int64_t* ns, int32_t n_n, uint32_t kmax, int32_t n_seeds,
                              uint64_t seed0, int64_t replicates, const uint32_t* q_num,
                              const uint32_t* q_den, int32_t n_q, double* table_out,
                              double* per_run_out, void* stream) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  if (!gammas || !ns || n_gamma < 1 || n_n < 1)
    return fail(ZPL_EINVAL, "need at least one exponent and one sample size");
  if ((int64_t)n_gamma * n_n > ((int64_t)1 << 20))
    return fail(ZPL_EINVAL, "table of %d x %d entries is too large", n_n, n_gamma);
  if (n_seeds < 1 || n_seeds > 1024)
    return fail(ZPL_EINVAL, "n_seeds must be in [1, 1024], got %d", n_seeds);
  if (n_q < 1 || !q_num || !q_den || !table_out)
    return fail(ZPL_EINVAL, "need at least one quantile and table_out");
  HIP_TRY(hipSetDevice(c->device));
  const hipStream_t s = (hipStream_t)stream;
  // the runs in entry-major order: (i_n, i_g, s)
  const int64_t n_runs = (int64_t)n_n * n_gamma * n_seeds;
  std::vector<zpl_cell> runs((size_t)n_runs);
  for (int in = 0; in < n_n; ++in)
    for (int ig = 0; ig < n_gamma; ++ig)
      for (int sd = 0; sd < n_seeds; ++sd) {
        zpl_cell& z = runs[((size_t)in * n_gamma + ig) * n_seeds + sd];
        z.alpha = gammas[ig];
        z.n = ns[in];
        z.replicates = replicates;
        z.seed = seed0 + (uint64_t)sd;
        z.stream = (uint32_t)(in * n_gamma + ig);
        z.kmax = kmax;
      }
  // groups of whole runs whose D values, selection scratch and tables fit in
  // a quarter of the budget (at least one run per group)
  const int64_t per_run = replicates * 8 +
                          (int64_t)kSelQ * (std::min<int64_t>(kSelGather, replicates * 3 / 20 + 1024) * 8 + 32) +
                          (int64_t)kH * 8 + (int64_t)(kGuide + 1) * 2;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>((int64_t)(c->budget / 4) / per_run, 4096));
  std::vector<double> q((size_t)n_runs * n_q);
  for (int64_t r0 = 0; r0 < n_runs; r0 += cap) {
    const int nr = (int)std::min<int64_t>(cap, n_runs - r0);
    Outputs out{nullptr, nullptr, nullptr, nullptr, nullptr};
    ZPL_TRY(run_cells(c, runs.data() + r0, nr, q_num, q_den, n_q, q.data() + r0 * n_q, out,
                      nullptr, s));
  }
  for (int64_t e = 0; e < (int64_t)n_n * n_gamma; ++e)
    for (int k = 0; k < n_q; ++k) {
      double sum = 0.0;
      for (int sd = 0; sd < n_seeds; ++sd) sum += q[((size_t)e * n_seeds + sd) * n_q + k];
      table_out[e * n_q + k] = sum / (double)n_seeds;
    }
  if (per_run_out) std::memcpy(per_run_out, q.data(), sizeof(double) * q.size());
  return ZPL_OK;
}

zpl_status zpl_autotune(zpl_ctx* c, const double* alphas, int32_t n_alpha, const int64_t* ns,
                        int32_t n_n, zpl_tune_entry* table_out, void* stream) {
  g_err.clear();
  if (!c || !alphas || !ns) return fail(ZPL_EINVAL, "NULL argument");
  if (n_alpha < 1 || n_n < 1 || n_alpha > kTuneMaxAxis || n_n > kTuneMaxAxis)
    return fail(ZPL_EINVAL, "grid axes need 1..%d values", kTuneMaxAxis);
  for (int i = 0; i < n_alpha; ++i) {
    if (!(alphas[i] >= kMinAlpha) || !(alphas[i] <= 64.0))
      return fail(ZPL_EINVAL, "alpha %g outside [1.01, 64]", alphas[i]);
    if (i > 0 && !(alphas[i] > alphas[i - 1])) return fail(ZPL_EINVAL, "alphas must increase");
  }
  for (int i = 0; i < n_n; ++i) {
    if (ns[i] < 1 || ns[i] > ((int64_t)1 << 20))
      return fail(ZPL_EINVAL, "grid n %lld outside [1, 2^20]", (long long)ns[i]);
    if (i > 0 && !(ns[i] > ns[i - 1])) return fail(ZPL_EINVAL, "ns must increase");
  }
  HIP_TRY(hipSetDevice(c->device));
  std::vector<zpl_tune_entry> tab;
  ZPL_TRY(autotune_grid(c, alphas, n_alpha, ns, n_n, tab, (hipStream_t)stream));
  ZPL_TRY(parse_tuning(tab.data(), (int32_t)tab.size(), c->tune));
  if (table_out) std::memcpy(table_out, tab.data(), sizeof(zpl_tune_entry) * tab.size());
  return ZPL_OK;
}

zpl_status zpl_set_tuning(zpl_ctx* c, const zpl_tune_entry* table, int32_t count) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  Tuning t;
  ZPL_TRY(parse_tuning(table, count, t));
  c->tune = std::move(t);
  return ZPL_OK;
}

zpl_status zpl_plan_forms(const zpl_tune_entry* table, int32_t count, const zpl_cell* cells,
                          int32_t n_cells, int32_t* forms_out) {
  g_err.clear();
  if (n_cells < 1 || !cells || !forms_out) return fail(ZPL_EINVAL, "need cells and forms_out");
  Tuning t;
  ZPL_TRY(parse_tuning(table, count, t));
  Plan P;
  ZPL_TRY(make_plan(cells, n_cells, ZPL_FORM_AUTO, P, &t));
  for (int i = 0; i < n_cells; ++i) forms_out[i] = (int32_t)P.cells[i].mode + 1;
  return ZPL_OK;
}

zpl_status zpl_set_timing(zpl_ctx* c, int32_t enable) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  c->timing = enable != 0;
  return ZPL_OK;
}

zpl_status zpl_get_timing(zpl_ctx* c, double* ms4) {
  g_err.clear();
  if (!c || !ms4) return fail(ZPL_EINVAL, "NULL argument");
  if (!c->timed) return fail(ZPL_EINVAL, "no timed simulation since timing was enabled");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipEventSynchronize(c->ev[4]));
  for (int k = 0; k < 4; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
    ms4[k] = (double)ms;
  }
  return ZPL_OK;
}

zpl_status zpl_fit(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                   double* alpha_hat, double* D, uint32_t* flags, void* stream) {
  g_err.clear();
  if (!c || !x || !alpha_hat || !D || !flags) return fail(ZPL_EINVAL, "NULL argument");
  if (n < 1 || n > ((int64_t)1 << 31)) return fail(ZPL_EINVAL, "n must be in [1, 2^31]");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t* xd;
  ZPL_TRY(stage_x(c, x, n, x_on_device, s, &xd));
  uint32_t st = 0;
  ZPL_TRY(fit_device(c, xd, n, s, alpha_hat, D, flags, &st));
  if (st & kErrBadValue) return fail(ZPL_EINVAL, "every x must be >= 1");
  if (*flags & ZPL_FLAG_NOCONV) return fail(ZPL_ENOCONV, "MLE iteration cap reached");
  return ZPL_OK;
}

zpl_status zpl_fit_noalloc(zpl_ctx* c, const int64_t* x_dev, int64_t n, uint32_t kmax,
                           double* alpha_hat_dev, double* D_dev, uint32_t* flags_dev,
                           uint32_t* status_dev, void* stream) {
  g_err.clear();
  if (!c || !x_dev || !alpha_hat_dev || !D_dev || !flags_dev || !status_dev)
    return fail(ZPL_EINVAL, "NULL argument");
  if (n < 1 || n > kNoAllocMaxN)
    return fail(ZPL_EINVAL, "n must be in [1, %lld] (the fixed scratch of the allocation-free "
                "fit holds one dataset of at most that size), got %lld",
                (long long)kNoAllocMaxN, (long long)n);
  if (kmax != 0 && (kmax < 2 || kmax > (uint32_t)kH))
    return fail(ZPL_EINVAL, "kmax must be 0 or in [2, %d], got %u", kH, kmax);
  const int64_t stride = heavy_stride(n);
  if (stride > kNoAllocStride)
    return fail(ZPL_EINVAL, "dataset of %lld values needs %lld scratch words, more than the "
                "fixed %lld", (long long)n, (long long)stride, (long long)kNoAllocStride);
  HIP_TRY(hipSetDevice(c->device));
  // the workgroup fit gives the same bits as the one-wave fit at every n
  HIP_TRY(launch_fit_block(x_dev, n, c->ln, c->noalloc_scratch, stride, alpha_hat_dev, D_dev,
                           flags_dev, status_dev, kmax, (hipStream_t)stream));
  return ZPL_OK;
}

zpl_status zpl_fit_scan(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                        const int64_t* xmins, int32_t n_xmin, double* alpha_hat, double* D,
                        int64_t* n_tail, uint32_t* flags, int32_t* best, void* stream) {
  g_err.clear();
  if (!c || !x || !xmins || !alpha_hat || !D || !n_tail || !flags || !best)
    return fail(ZPL_EINVAL, "NULL argument");
  if (n < 1 || n > ((int64_t)1 << 31)) return fail(ZPL_EINVAL, "n must be in [1, 2^31]");
  if (n_xmin < 1 || n_xmin > 65536) return fail(ZPL_EINVAL, "n_xmin must be in [1, 65536]");
  for (int i = 0; i < n_xmin; ++i)
    if (xmins[i] < 1 || xmins[i] > kMaxXmin)
      return fail(ZPL_EINVAL, "candidate %d: xmin must be in [1, 2^40], got %lld", i,
                  (long long)xmins[i]);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t* xd;
  ZPL_TRY(stage_x(c, x, n, x_on_device, s, &xd));
  // one wave per candidate; each wave keeps its overflow and list areas in
  // the heavy scratch, so the grid is what a quarter of the budget holds
  const int64_t stride = heavy_stride(n);
  int grid = std::min(n_xmin, 4 * c->n_cu);
  while (grid > 1 && (uint64_t)grid * stride * 8 > c->budget / 4) grid /= 2;
  const size_t nc = (size_t)n_xmin;
  ZPL_TRY(ensure(c, c->heavy, sizeof(int64_t) * (size_t)stride * grid));
  ZPL_TRY(ensure(c, c->scan, nc * (sizeof(int64_t) + 2 * sizeof(double) + sizeof(int64_t) +
                                   2 * sizeof(uint32_t))));
  const size_t host_bytes = nc * (2 * sizeof(double) + sizeof(int64_t) + 2 * sizeof(uint32_t));
  ZPL_TRY(ensure_pinned(c, std::max(host_bytes, nc * sizeof(int64_t))));
  HIP_TRY(hipStreamSynchronize(s));  // the staging area may still be in use
  std::memcpy(c->pin, xmins, nc * sizeof(int64_t));
  char* dp = (char*)c->scan.p;
  int64_t* d_xmins = (int64_t*)dp;
  double* d_a = (double*)(dp + nc * 8);
  double* d_D = d_a + nc;
  int64_t* d_nt = (int64_t*)(d_D + nc);
  uint32_t* d_fl = (uint32_t*)(d_nt + nc);
  uint32_t* d_st = d_fl + nc;
  HIP_TRY(hipMemcpyAsync(d_xmins, c->pin, nc * sizeof(int64_t), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_fit_scan(grid, xd, n, d_xmins, n_xmin, c->ln, (int64_t*)c->heavy.p, stride,
                          d_a, d_D, d_nt, d_fl, d_st, s));
  // results: alpha_hat, D, n_tail, flags, status are contiguous on the device
  HIP_TRY(hipMemcpyAsync(c->pin, d_a, host_bytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const char* hp = (const char*)c->pin;
  std::memcpy(alpha_hat, hp, nc * 8);
  std::memcpy(D, hp + nc * 8, nc * 8);
  std::memcpy(n_tail, hp + nc * 16, nc * 8);
  std::memcpy(flags, hp + nc * 24, nc * 4);
  const uint32_t* st = (const uint32_t*)(hp + nc * 28);
  int b = -1;
  for (int i = 0; i < n_xmin; ++i) {
    if (st[i] & kErrBadValue) return fail(ZPL_EINVAL, "every x must be >= 1");
    if (st[i] & kErrNoTail) continue;
    if (b < 0 || D[i] < D[b]) b = i;
  }
  *best = b;
  return ZPL_OK;
}

zpl_status zpl_fit_xmin(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                        int64_t xmin, double* alpha_hat, double* D, int64_t* n_tail,
                        uint32_t* flags, void* stream) {
  int32_t best = -1;
  ZPL_TRY(zpl_fit_scan(c, x, n, x_on_device, &xmin, 1, alpha_hat, D, n_tail, flags, &best,
                       stream));
  if (best < 0) return fail(ZPL_EINVAL, "no value is >= xmin = %lld", (long long)xmin);
  if (*flags & ZPL_FLAG_NOCONV) return fail(ZPL_ENOCONV, "the MLE root lies above 64");
  return ZPL_OK;
}

zpl_status zpl_fit_truncated(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                             uint32_t kmax, double* alpha_hat, double* D, uint32_t* flags,
                             void* stream) {
  g_err.clear();
  if (!c || !x || !alpha_hat || !D || !flags) return fail(ZPL_EINVAL, "NULL argument");
  if (n < 1 || n > ((int64_t)1 << 31)) return fail(ZPL_EINVAL, "n must be in [1, 2^31]");
  if (kmax < 2 || kmax > (uint32_t)kH)
    return fail(ZPL_EINVAL, "kmax must be in [2, %d], got %u", kH, kmax);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t* xd;
  ZPL_TRY(stage_x(c, x, n, x_on_device, s, &xd));
  uint32_t st = 0;
  ZPL_TRY(fit_device(c, xd, n, s, alpha_hat, D, flags, &st, kmax));
  if (st & kErrBadValue) return fail(ZPL_EINVAL, "every x must be in [1, %u]", kmax);
  if (*flags & ZPL_FLAG_NOCONV)
    return fail(ZPL_ENOCONV, "the mean log has no root in [-64, 64] (or the iteration cap was reached)");
  return ZPL_OK;
}

zpl_status zpl_bootstrap_pvalue(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                                int64_t B, uint64_t seed, uint32_t stream_id,
                                double* alpha_hat, double* D, double* p_value,
                                uint32_t* flags, void* stream) {
  g_err.clear();
  if (!c || !x || !alpha_hat || !D || !p_value || !flags)
    return fail(ZPL_EINVAL, "NULL argument");
  if (B < 1 || B > ((int64_t)1 << 32)) return fail(ZPL_EINVAL, "B must be in [1, 2^32]");
  zpl_status st = zpl_fit(c, x, n, x_on_device, alpha_hat, D, flags, stream);
  if (st != ZPL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  zpl_cell cell = {*alpha_hat, n, B, seed, stream_id, 0};
  ZPL_TRY(ensure(c, c->boot_d, sizeof(double) * (size_t)B + 64));
  ZPL_TRY(ensure(c, c->count, sizeof(unsigned long long) + sizeof(double)));
  Outputs out{(double*)c->boot_d.p, nullptr, nullptr, nullptr, nullptr};
  ZPL_TRY(run_cells(c, &cell, 1, nullptr, nullptr, 0, nullptr, out, nullptr, s));
  // D_obs to the device, count D_b >= D_obs
  ZPL_TRY(ensure_pinned(c, 64));
  HIP_TRY(hipStreamSynchronize(s));
  double* pd = (double*)c->pin;
  pd[0] = *D;
  unsigned long long* cnt = (unsigned long long*)c->count.p;
  double* dobs = (double*)(cnt + 1);
  HIP_TRY(hipMemcpyAsync(dobs, pd, sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_fill_u32((uint32_t*)cnt, 2, 0u, s));
  HIP_TRY(launch_count_ge((const double*)c->boot_d.p, B, dobs, cnt, s));
  unsigned long long* hc = (unsigned long long*)((char*)c->pin + 8);
  HIP_TRY(hipMemcpyAsync(hc, cnt, sizeof *hc, hipMemcpyDeviceToHost, s));
  ZPL_TRY(check_err_word(c, s));
  *p_value = (double)*hc / (double)B;
  return ZPL_OK;
}

zpl_status zpl_serve_start(zpl_ctx* c, const zpl_serve_opts* opts) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  if (c->server) return fail(ZPL_EINVAL, "serving already started on this context");
  zpl_serve_opts o = {0, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.reserved2 != 0) return fail(ZPL_EINVAL, "opts.reserved2 must be 0");
  if (o.slice_us < 0 || o.max_batch < 0 || o.max_queue < 0)
    return fail(ZPL_EINVAL, "opts: negative slice_us, max_batch or max_queue");
  Server* sv = new Server();
  if (o.mem_budget_bytes) sv->budget = o.mem_budget_bytes;
  if (sv->budget > c->budget) {
    const unsigned long long b = sv->budget, cb = c->budget;
    delete sv;
    return fail(ZPL_EINVAL, "serving budget %llu exceeds the context's budget %llu", b, cb);
  }
  if (o.max_batch > 0) sv->max_active = o.max_batch;
  if (o.max_queue > 0) sv->max_queue = o.max_queue;
  if (o.slice_us > 0) sv->slice_ns = 1e3 * (double)o.slice_us;
  zpl_status st = zpl_create(&sv->eng, c->device, c->budget);
  if (st != ZPL_OK) {
    delete sv;
    return st;
  }
  sv->eng->tune = c->tune;
  if (hipStreamCreateWithFlags(&sv->submit_stream, hipStreamNonBlocking) != hipSuccess) {
    zpl_destroy(sv->eng);
    delete sv;
    return fail(ZPL_EDEVICE, "serving: could not create the submit stream");
  }
  sv->th = std::thread([sv] { sv->loop(); });
  c->server = sv;
  return ZPL_OK;
}

zpl_status zpl_serve_submit(zpl_ctx* c, const int64_t* x, int64_t n, int32_t x_on_device,
                            int64_t B, uint64_t seed, uint32_t stream_id, uint64_t* ticket) {
  g_err.clear();
  if (!c || !x || !ticket) return fail(ZPL_EINVAL, "NULL argument");
  Server* sv = c->server;
  if (!sv) return fail(ZPL_EINVAL, "serving not started");
  if (n < 1 || n > ((int64_t)1 << 31)) return fail(ZPL_EINVAL, "n must be in [1, 2^31]");
  if (B < 1 || B > ((int64_t)1 << 32)) return fail(ZPL_EINVAL, "B must be in [1, 2^32]");
  Req* r = new Req();
  r->n = n;
  if (x_on_device) {
    // a device copy that stays on the device until the request's fit
    HIP_TRY(hipSetDevice(c->device));
    const size_t bytes = sizeof(int64_t) * (size_t)n;
    hipError_t e = hipMallocAsync((void**)&r->xdev, bytes, sv->submit_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r->xdev, x, bytes, hipMemcpyDeviceToDevice, sv->submit_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->submit_stream);
    if (e != hipSuccess) {
      if (r->xdev) (void)hipFree(r->xdev);
      delete r;
      return fail(e == hipErrorOutOfMemory ? ZPL_ENOMEM : ZPL_EDEVICE,
                  "serving: device dataset copy: %s", hipGetErrorString(e));
    }
  } else {
    r->x.assign(x, x + n);
  }
  r->B = B;
  r->seed = seed;
  r->stream_id = stream_id;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->fatal.empty() || (int)sv->queue.size() >= sv->max_queue) {
      if (r->xdev) (void)hipFreeAsync(r->xdev, sv->submit_stream);
      delete r;
      if (!sv->fatal.empty()) return fail(ZPL_EDEVICE, "%s", sv->fatal.c_str());
      return fail(ZPL_EBUSY, "serving queue full (%d requests)", sv->max_queue);
    }
    r->ticket = sv->next_ticket++;
    sv->reqs[r->ticket] = r;
    sv->queue.push_back(r);
  }
  sv->cv.notify_all();
  *ticket = r->ticket;
  return ZPL_OK;
}

zpl_status zpl_serve_poll(zpl_ctx* c, uint64_t ticket, int32_t wait_ms, zpl_serve_result* res) {
  g_err.clear();
  if (!c || !res) return fail(ZPL_EINVAL, "NULL argument");
  Server* sv = c->server;
  if (!sv) return fail(ZPL_EINVAL, "serving not started");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(ZPL_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second;
  if (!r->done && wait_ms > 0)
    sv->cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return r->done; });
  std::memset(res, 0, sizeof *res);
  res->done = r->done ? 1 : 0;
  if (!r->done) return ZPL_OK;
  res->status = r->status;
  res->alpha_hat = r->ahat;
  res->D = r->D;
  res->p_value = r->p;
  res->flags = r->flags;
  res->batch_size = r->mix;
  res->launches = r->launches;
  using ms = std::chrono::duration<double, std::milli>;
  res->queue_ms = ms(r->t_start - r->t_submit).count();
  res->latency_ms = ms(r->t_done - r->t_submit).count();
  sv->reqs.erase(it);
  delete r;
  return ZPL_OK;
}

zpl_status zpl_serve_stop(zpl_ctx* c) {
  g_err.clear();
  if (!c) return fail(ZPL_EINVAL, "ctx is NULL");
  Server* sv = c->server;
  if (!sv) return ZPL_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  for (auto& kv : sv->reqs) {
    if (kv.second->xdev) (void)hipFreeAsync(kv.second->xdev, sv->submit_stream);
    delete kv.second;
  }
  if (sv->submit_stream) {
    (void)hipStreamSynchronize(sv->submit_stream);
    (void)hipStreamDestroy(sv->submit_stream);
  }
  zpl_destroy(sv->eng);
  delete sv;
  c->server = nullptr;
  return ZPL_OK;
}

zpl_status zpl_sample_draws(zpl_ctx* c, double alpha, uint32_t kmax, int64_t xmin, int64_t n,
                            uint64_t seed, uint32_t stream_id, int64_t rep_lo, int64_t count,
                            int64_t* x_out, uint32_t* flags_out, void* stream) {
  g_err.clear();
  if (!c || !x_out || !flags_out) return fail(ZPL_EINVAL, "NULL argument");
  if (n < 1 || count < 1 || rep_lo < 0 || rep_lo + count > ((int64_t)1 << 32) ||
      n > ((int64_t)1 << 31))
    return fail(ZPL_EINVAL, "bad n / replicate range");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  zpl_cell z = {alpha, n, count, seed, stream_id, kmax, xmin};
  Plan P;
  ZPL_TRY(make_plan(&z, 1, ZPL_FORM_HEAVY, P));  // validates alpha, kmax and xmin
  ZPL_TRY(ensure(c, c->plan, sizeof(DevCell)));
  ZPL_TRY(ensure(c, c->tables, sizeof(double) * kH));
  ZPL_TRY(ensure(c, c->guides, sizeof(uint16_t) * (kGuide + 1)));
  ZPL_TRY(ensure_pinned(c, sizeof(DevCell)));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(c->pin, &P.cells[0], sizeof(DevCell));
  HIP_TRY(hipMemcpyAsync(c->plan.p, c->pin, sizeof(DevCell), hipMemcpyHostToDevice, s));
  ++c->plan_gen;
  HIP_TRY(launch_tables((DevCell*)c->plan.p, 1, (double*)c->tables.p, (uint16_t*)c->guides.p,
                        c->ln, s, z.kmax != 0));
  HIP_TRY(launch_fill_u32(flags_out, (int)count, 0u, s));
  HIP_TRY(launch_draws((const DevCell*)c->plan.p, (const double*)c->tables.p,
                       (const uint16_t*)c->guides.p, rep_lo, count, x_out, flags_out,
                       count * n, s));
  return ZPL_OK;
}

zpl_status zpl_cdf_table(zpl_ctx* c, double alpha, uint32_t kmax, int64_t xmin, double* T_out,
                         void* stream) {
  g_err.clear();
  if (!c || !T_out) return fail(ZPL_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  zpl_cell z = {alpha, 1, 1, 0, 0, kmax, xmin};
  Plan P;
  ZPL_TRY(make_plan(&z, 1, ZPL_FORM_HEAVY, P));  // validates alpha, kmax and xmin
  ZPL_TRY(ensure(c, c->plan, sizeof(DevCell)));
  ZPL_TRY(ensure(c, c->tables, sizeof(double) * kH));
  ZPL_TRY(ensure(c, c->guides, sizeof(uint16_t) * (kGuide + 1)));
  ZPL_TRY(ensure_pinned(c, sizeof(DevCell)));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(c->pin, &P.cells[0], sizeof(DevCell));
  HIP_TRY(hipMemcpyAsync(c->plan.p, c->pin, sizeof(DevCell), hipMemcpyHostToDevice, s));
  ++c->plan_gen;
  HIP_TRY(launch_tables((DevCell*)c->plan.p, 1, (double*)c->tables.p, (uint16_t*)c->guides.p,
                        c->ln, s, z.kmax != 0));
  HIP_TRY(hipMemcpyAsync(T_out, c->tables.p, sizeof(double) * kH, hipMemcpyDeviceToDevice, s));
  return ZPL_OK;
}

}  // extern "C"
