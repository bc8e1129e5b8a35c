// zpl_kernels.hip -- gfx950 kernels of the Zipf (xmin = 1) MLE + KS Monte
// Carlo path of Rappos & Robert (2013): CDF/guide table build, the replicate
// kernels (lane, wave and heavy forms), the dataset fit, order-statistic
// selection, and the bootstrap count.
//
// Per replicate (Sect. 3/4 of the paper): n draws from eq. (1) by inverse CDF
// with a Philox4x32-10 counter stream, S = sum ln x (exact 128-bit fixed
// point), alpha_hat from eq. (2), D from eq. (3) over the distinct values.
// None of this is a dense contraction: the kernels are VALU/LDS work laid out
// for wave64, with LDS-resident tables and histograms.
#include <hip/hip_runtime.h>

#include "zpl_kernels.hpp"
#include "zpl_math.hpp"

namespace zpl {

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) {
  return (uint32_t)__shfl_xor((int)v, m, 64);
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = shfl_xor_u32((uint32_t)v, m);
  const uint32_t hi = shfl_xor_u32((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += shfl_xor_u32(v, m);
  return v;
}
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v |= shfl_xor_u32(v, m);
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += shfl_xor_u64(v, m);
  return v;
}
__device__ __forceinline__ int64_t wave_max_i64(int64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const int64_t o = (int64_t)shfl_xor_u64((uint64_t)v, m);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ U128 wave_sum_u128(U128 v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const uint64_t lo = shfl_xor_u64(v.lo, m);
    const uint64_t hi = shfl_xor_u64(v.hi, m);
    u128_add(v, lo, hi);
  }
  return v;
}
__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Inverse-CDF sampling: x = min{k in 1..kH : T[k] >= U} (the ">=" rule of
// the paper's sampler).  U = m 2^-53 with m = (w >> 11) | 1 an odd 53-bit
// integer, and the LDS copy of the table holds TI[k] = floor(T[k] 2^53), so
// T[k] >= U exactly when TI[k] >= m: every comparison is a 64-bit integer
// one and U is never formed.  The guide brackets the answer in
// [g[b], g[b+1]]; most brackets are one or two values wide, resolved with at
// most one table probe ("fast path").  Wider brackets and U > T[kH] (the
// tail) are deferred and resolved 64 at a time.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t m53(uint32_t hi, uint32_t lo) {
  return ((((uint64_t)hi) << 32 | (uint64_t)lo) >> 11) | 1ull;
}

// Packed guide entry (guide_pack): the draw is lo when TI[lo] >= m (a
// bracket [lo, lo] always has it); otherwise the high half, which is hi when
// that is the answer, else >= kDeferred: the draw is deferred (a wider
// bracket, or a tail uniform m > TI[kH], which never has TI[lo] >= m).
// Every m indexes a valid guide entry and 1 <= lo <= kH.
__device__ __forceinline__ int fast_select(uint32_t gg, uint64_t ti, uint64_t m) {
  return ti >= m ? (int)(gg & 0xffffu) : (int)(gg >> 16);
}

__device__ __forceinline__ int fast_draw(uint64_t m, const uint64_t* __restrict__ T,
                                         const uint32_t* __restrict__ guide, int sh) {
  const uint32_t gg = guide[guide_index(m, sh)];
  uint64_t ti = T[(int)(gg & 0xffffu) - 1];
  asm volatile("" : "+v"(ti));  // keep the read unconditional (no divergent branch)
  return fast_select(gg, ti, m);
}

// fast_draw for four draws at once, in phases (all guide reads, then all
// table reads, then the selections) so that the reads of each phase are in
// flight together: two LDS round trips per four draws instead of eight.
__device__ __forceinline__ void fast_draw4(const uint64_t (&m)[4], const uint64_t* __restrict__ T,
                                           const uint32_t* __restrict__ guide, int sh,
                                           int (&x)[4]) {
  uint32_t gg[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) gg[d] = guide[guide_index(m[d], sh)];
  uint64_t t[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) t[d] = T[(int)(gg[d] & 0xffffu) - 1];
  asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]));  // reads stay unconditional
#pragma unroll
  for (int d = 0; d < 4; ++d) x[d] = fast_select(gg[d], t[d], m[d]);
}

// Full search of a deferred body draw.
__device__ __forceinline__ int slow_search(uint64_t m, const uint64_t* __restrict__ T,
                                           const uint32_t* __restrict__ guide, int sh) {
  const uint32_t gg = guide[guide_index(m, sh)];
  int lo = (int)(gg & 0xffffu), hi = (int)((gg >> 16) & (kDeferred - 1));
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (T[mid - 1] >= m)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}


// Deferred draw of the lane and wave forms in 8 bytes.  Bit 63 clear: a body
// draw, bits 0..52 = m.  Bit 63 set: a tail draw, bits 0..31 = its index in
// the replicate.  Bits 53..58: the lane that owns the replicate (lane form).
__device__ __forceinline__ uint64_t defer_entry(uint64_t m, uint64_t timax, uint32_t i, int owner) {
  const uint64_t o = (uint64_t)owner << 53;
  return m > timax ? ((1ull << 63) | o | i) : (o | m);
}



// ---------------------------------------------------------------------------
// KS distance (eq. 3) over the distinct values of one replicate, in
// ascending order.  With C the count of draws <= t and Z(t) = zeta(a, t+1)
// (so F(t) = 1 - Z(t)/zeta(a)), each distinct value v contributes
// |Z(v)/zeta - (n - C(v))/n| and |Z(v-1)/zeta - (n - C(v-1))/n|: between
// sample values S_n is flat and F rises, so the sup over all t is reached at
// a sample value or one below it.  Values <= 16 use the precomputed head
// suf[]; for larger ones Z(v) comes from the Euler-Maclaurin tail and
// Z(v-1) = Z(v) + v^-a.  Src yields the distinct values: small(v) returns
// the count of v for v = 1..16 in order, then next_large() returns the
// remaining (value, count) pairs ascending.
// ---------------------------------------------------------------------------
template <class Src>
__device__ __forceinline__ double ks_distance(Src& src, const EmCoef& E,
                                              const double (&suf)[17], int64_t n,
                                              const double* __restrict__ ln) {
  const double iz = 1.0 / suf[0], idn = 1.0 / (double)n;
  int64_t C = 0;
  double D = 0.0;
#pragma unroll
  for (int v = 1; v <= 16; ++v) {
    const uint32_t c = src.small(v);
    if (c) {
      const double t2 = fabs(fma(suf[v - 1], iz, -(double)(n - C) * idn));
      C += c;
      const double t1 = fabs(fma(suf[v], iz, -(double)(n - C) * idn));
      D = fmax(D, fmax(t1, t2));
    }
  }
  double zprev = suf[16];
  int64_t vprev = 16;
  // The table logarithms ln v and ln(v + 1) of each entry are read one entry
  // ahead (at indexes clamped into the table; values past it take log), so
  // their latency overlaps the previous entry's arithmetic.
  constexpr int64_t kLnTop = (int64_t)kH + 1;
  int64_t v = 0;
  uint32_t c = 0;
  bool have = src.next_large(v, c);
  double lv = ln[v < kLnTop ? v : kLnTop], lv1 = ln[v < kLnTop ? v + 1 : kLnTop];
  while (have) {
    int64_t vn = 0;
    uint32_t cn = 0;
    const bool haven = src.next_large(vn, cn);
    const double lvn = ln[vn < kLnTop ? vn : kLnTop];
    const double lvn1 = ln[vn < kLnTop ? vn + 1 : kLnTop];
    // survival_next and ln_value with the logarithms read ahead
    const double q = (double)v + 1.0;
    const double zv = hurwitz_tail(E, q, v < kLnTop ? lv1 : log(q));
    const double zv1 =
        (v - 1 == vprev) ? zprev : zv + pow_neg(E.s, v <= kLnTop ? lv : log((double)v));
    const double t2 = fabs(fma(zv1, iz, -(double)(n - C) * idn));
    C += c;
    const double t1 = fabs(fma(zv, iz, -(double)(n - C) * idn));
    D = fmax(D, fmax(t1, t2));
    zprev = zv;
    vprev = v;
    v = vn;
    c = cn;
    lv = lvn;
    lv1 = lvn1;
    have = haven;
  }
  return D;
}

// KS distance (eq. 3) under the truncated law on 1..K: F(t) = P(t)/Z with
// P(t) = sum_{k<=t} k^-a accumulated in ascending k as the distinct values
// are visited, and Z = Z_K(a) (zeta3_trunc_fast: Euler-Maclaurin for large
// K, else the K terms from K down).  Same terms as
// ks_distance: |F(v) - C(v)/n| and |F(v-1) - C(v-1)/n| per distinct v.
template <class Src>
__device__ __forceinline__ double ks_distance_trunc(Src& src, double a, uint32_t K, int64_t n,
                                                    const double* __restrict__ ln) {
  const double Z = zeta3_trunc_fast(a, K, ln).z0;  // the normaliser Z_K(a)
  const double iz = 1.0 / Z, idn = 1.0 / (double)n;
  int64_t C = 0;
  double D = 0.0, P = 0.0;
  int64_t k = 0;  // P = P(k)
  auto term = [&](int64_t v, uint32_t c) {
    while (k < v - 1) {
      ++k;
      P += k == 1 ? 1.0 : pow_neg(a, ln[k]);
    }
    const double t2 = fabs(fma(P, iz, -(double)C * idn));
    ++k;
    P += k == 1 ? 1.0 : pow_neg(a, ln[k]);
    C += c;
    const double t1 = fabs(fma(P, iz, -(double)C * idn));
    D = fmax(D, fmax(t1, t2));
  };
#pragma unroll
  for (int v = 1; v <= 16; ++v) {
    const uint32_t c = src.small(v);
    if (c) term(v, c);
  }
  int64_t v;
  uint32_t c;
  while (src.next_large(v, c)) term(v, c);
  return D;
}

// S (with the paper's all-ones rule), alpha_hat (eq. 2) and D (eq. 3), for
// the pure law (K = 0) or the truncated law on 1..K.
template <class Src>
__device__ __forceinline__ void finish_replicate(Src& src, const U128& S, int64_t n,
                                                 uint32_t fl, const double* __restrict__ ln,
                                                 uint32_t K, double& ahat, double& D,
                                                 uint32_t& flags) {
  double Sd;
  if (S.lo == 0 && S.hi == 0) {  // every draw was 1: S := ln 2
    Sd = ln[2];
    fl |= kFlagAllOnes;
  } else {
    Sd = u128_to_S(S);
  }
  if (K) {
    const double a = mle_alpha_trunc(Sd / (double)n, K, ln, &fl);
    D = ks_distance_trunc(src, a, K, n, ln);
    ahat = a;
  } else {
    const double a = mle_alpha(Sd / (double)n, ln, &fl);
    const EmCoef E = em_coef(a);
    double suf[17];
    survival_head(E, ln, suf);
    D = ks_distance(src, E, suf, n, ln);
    ahat = a;
  }
  flags = fl;
}

__device__ __forceinline__ void write_outputs(const Outputs& o, int64_t idx, double D,
                                              double a, uint32_t fl, uint64_t fp,
                                              int64_t xmax) {
  if (o.D) o.D[idx] = D;
  if (o.ahat) o.ahat[idx] = a;
  if (o.flags) o.flags[idx] = fl;
  if (o.fp) o.fp[idx] = fp;
  if (o.xmax) o.xmax[idx] = xmax;
}

// ---------------------------------------------------------------------------
// Distinct-value sources.
// ---------------------------------------------------------------------------
// Lane mode: a per-lane column of packed 16-bit counters for values 1..kHLB
// (dword b holds values 2b+1 and 2b+2) and a sorted per-lane overflow list.
struct LaneSrc {
  const uint32_t* hist;  // element (b, lane) at hist[b * 64]
  const int64_t* ov;     // element (p, lane) at ov[p * 64]
  int oc;
  int bin;  // next value to inspect in 17..kHLB
  int p;    // next overflow index
  __device__ __forceinline__ uint32_t count(int v) const {
    const uint32_t w = hist[((v - 1) >> 1) * 64];
    return ((v - 1) & 1) ? (w >> 16) : (w & 0xffffu);
  }
  __device__ __forceinline__ uint32_t small(int v) { return count(v); }
  __device__ __forceinline__ bool next_large(int64_t& v, uint32_t& c) {
    while (bin <= kHLB) {
      const int b = bin++;
      const uint32_t k = count(b);
      if (k) {
        v = b;
        c = k;
        return true;
      }
    }
    if (p < oc) {
      const int64_t x = ov[p * 64];
      uint32_t k = 0;
      while (p < oc && ov[p * 64] == x) {
        ++p;
        ++k;
      }
      v = x;
      c = k;
      return true;
    }
    return false;
  }
};

// A compact ascending (value, count) list in global memory.  The entry after
// the one being consumed is loaded ahead, so its latency overlaps the FP64
// work of the current value.
struct ListSrc {
  const int64_t* vals;
  const uint32_t* cnts;
  int len;
  int p;  // index of the entry held in (nv, nc)
  int64_t nv;
  uint32_t nc;
  __device__ __forceinline__ ListSrc(const int64_t* v, const uint32_t* c, int l)
      : vals(v), cnts(c), len(l), p(0), nv(0), nc(0u) {
    if (len > 0) {
      nv = vals[0];
      nc = cnts[0];
    }
  }
  __device__ __forceinline__ void advance() {
    ++p;
    if (p < len) {
      nv = vals[p];
      nc = cnts[p];
    }
  }
  __device__ __forceinline__ uint32_t small(int v) {
    if (p < len && nv == (int64_t)v) {
      const uint32_t c = nc;
      advance();
      return c;
    }
    return 0u;
  }
  __device__ __forceinline__ bool next_large(int64_t& v, uint32_t& c) {
    if (p >= len) return false;
    v = nv;
    c = nc;
    advance();
    return true;
  }
};

// ks_distance over a compact ascending list in global memory, by a whole
// wave: the values <= 16 are taken by every lane as in ks_distance, the rest
// is cut into 64 contiguous chunks, one per lane.  A wave prefix sum gives
// each chunk its count C of draws below it, and a chunk whose first value v
// follows its predecessor (v - 1 = previous value) recomputes the same
// zeta(a, v) the sequential loop would have carried over, so every term, and
// hence the maximum, is bit-identical to ks_distance.  Returns D on every lane.
__device__ __forceinline__ uint64_t wave_excl_scan_u64(uint64_t v, int lane) {
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 64);
    if (lane >= d) x += ((uint64_t)hi << 32) | lo;
  }
  return x - v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const uint64_t b = shfl_xor_u64((uint64_t)__double_as_longlong(v), m);
    v = fmax(v, __longlong_as_double((long long)b));
  }
  return v;
}

// iz = 1/zeta(a, xmin): F(t) = 1 - zeta(a, t+1) iz for t >= xmin - 1 (the
// first distinct value's lower term is then zero).  cut: the law with a lower
// cutoff, whose survival values above 16 come from survival_next_cut (there
// they are the normaliser's own scale, not a tail of zeta(a)); xrel > 0: a
// cutoff xrel above 17, every survival value (and iz) taken relative to
// xrel^-a (survival_rel).
__device__ double ks_distance_wave(const int64_t* __restrict__ lv, const uint32_t* __restrict__ lc,
                                   int len, const EmCoef& E, const double (&suf)[17], int64_t n,
                                   const double* __restrict__ ln, int lane, double iz,
                                   bool cut = false, int64_t xrel = 0) {
  const double idn = 1.0 / (double)n;
  int64_t C = 0;
  double D = 0.0;
  int p = 0;
  // the list's first 64 entries, one per lane, in one round of loads; the
  // values <= 16 (at most the first 16 entries) are then read across lanes
  // instead of by a chain of dependent global loads
  const int64_t hv = lane < len ? lv[lane] : INT64_MAX;
  const uint32_t hc = lane < len ? lc[lane] : 0u;
#pragma unroll
  for (int v = 1; v <= 16; ++v) {
    const int64_t pv = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(uint32_t)(hv >> 32), p, 64) << 32) |
                                 (uint32_t)__shfl((int)(uint32_t)hv, p, 64));
    if (p < len && pv == (int64_t)v) {
      const double t2 = fabs(fma(suf[v - 1], iz, -(double)(n - C) * idn));
      C += (uint32_t)__shfl((int)hc, p, 64);
      const double t1 = fabs(fma(suf[v], iz, -(double)(n - C) * idn));
      D = fmax(D, fmax(t1, t2));
      ++p;
    }
  }
  const int p16 = p;
  const int chunk = (len - p16 + 63) / 64;
  const int q0 = p16 + lane * chunk;
  const int q1 = min(q0 + chunk, len);
  uint64_t cs = 0;
  for (int q = q0; q < q1; ++q) cs += lc[q];
  C += (int64_t)wave_excl_scan_u64(cs, lane);
  if (q0 < q1) {
    int64_t vprev = q0 == p16 ? 16 : lv[q0 - 1];
    double zprev = suf[16];
    bool have = q0 == p16;  // zprev is zeta(a, vprev + 1)
    // the next entry is loaded before this one's arithmetic, so the load's
    // latency overlaps it
    int64_t v = lv[q0];
    uint32_t cv = lc[q0];
    for (int q = q0; q < q1; ++q) {
      const int qn = q + 1 < q1 ? q + 1 : q;
      const int64_t vn = lv[qn];
      const uint32_t cn = lc[qn];
      const double zv = xrel ? survival_rel(E, v, xrel)
                             : (cut ? survival_next_cut(E, v, ln) : survival_next(E, v, ln));
      double zv1;
      if (v - 1 == vprev)
        zv1 = have ? zprev
                   : (xrel ? survival_rel(E, vprev, xrel)
                           : (cut ? survival_next_cut(E, vprev, ln) : survival_next(E, vprev, ln)));
      else
        zv1 = zv + (xrel ? pow_rel(E.s, v, xrel) : pow_neg(E.s, ln_value(v, ln)));
      const double t2 = fabs(fma(zv1, iz, -(double)(n - C) * idn));
      C += cv;
      const double t1 = fabs(fma(zv, iz, -(double)(n - C) * idn));
      D = fmax(D, fmax(t1, t2));
      zprev = zv;
      vprev = v;
      have = true;
      v = vn;
      cv = cn;
    }
  }
  return wave_max_f64(D);
}

// finish_replicate by a whole wave over a global list (heavy form, fit):
// every lane solves the same MLE; the KS is split over the lanes.
__device__ __forceinline__ void finish_replicate_wave(const int64_t* lv, const uint32_t* lc, int len,
                                                      const U128& S, int64_t n, uint32_t fl,
                                                      const double* __restrict__ ln, int lane,
                                                      uint32_t K, double& ahat, double& D,
                                                      uint32_t& flags, int64_t xmin = 1) {
  if (K) {  // O(K) per replicate either way: every lane runs the same sequence
    ListSrc src(lv, lc, len);
    finish_replicate(src, S, n, fl, ln, K, ahat, D, flags);
    return;
  }
  if (xmin > 1) {  // the law with a lower cutoff (every value >= xmin)
    U128 Sx = S;
    if (len == 1 && lv[0] == xmin) {  // every value at the cutoff: one counts as xmin + 1
      Sx = U128{0, 0};
      u128_add_mul(Sx, (uint64_t)(n - 1), ln_fixed(xmin, ln));
      u128_add(Sx, ln_fixed(xmin + 1, ln), 0);
      fl |= kFlagAllOnes;
    }
    const double a = mle_alpha_hz(u128_to_S(Sx) / (double)n, xmin, ln, &fl);
    const EmCoef E = em_coef(a);
    double suf[17];
    survival_head_cut(E, ln, suf);
    double zx = 0.0;  // zeta(a, xmin) = suf[xmin - 1] (static indices: no scratch)
#pragma unroll
    for (int t = 1; t <= 16; ++t)
      if (xmin - 1 == t) zx = suf[t];
    // above 17 every value is: survival values relative to xmin^-a
    if (xmin > 17) zx = survival_rel(E, xmin - 1, xmin);
    D = ks_distance_wave(lv, lc, len, E, suf, n, ln, lane, 1.0 / zx, true, xmin > 17 ? xmin : 0);
    ahat = a;
    flags = fl;
    return;
  }
  double Sd;
  if (S.lo == 0 && S.hi == 0) {
    Sd = ln[2];
    fl |= kFlagAllOnes;
  } else {
    Sd = u128_to_S(S);
  }
  const double a = mle_alpha(Sd / (double)n, ln, &fl);
  const EmCoef E = em_coef(a);
  double suf[17];
  survival_head(E, ln, suf);
  D = ks_distance_wave(lv, lc, len, E, suf, n, ln, lane, 1.0 / suf[0]);
  ahat = a;
  flags = fl;
}

// ---------------------------------------------------------------------------
// Wave-cooperative helpers for the wave and heavy forms.
// ---------------------------------------------------------------------------
// Ordering of one wave's global-memory stores before its later loads.
__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Builds the compact (value, count) list of one replicate from a histogram
// of values 1..nbins (hist[v-1]) and a sorted overflow array ov[0..oc),
// appending at lv/lc (length returned).  Also returns, identical on every
// lane, the exact 128-bit sum of ln x and, when want_fp, the multiset
// fingerprint and the largest value.  The histogram is consumed: when every
// count fits in 21 bits (n < 2^21) its nonzero bins are also packed as
// (v << 21 | count) into hist[0..) in list order, so the sums read them from
// LDS instead of reading the global list back.
struct Summary {
  U128 S;
  uint64_t fp;
  int64_t xmax;
  int len;
};

__device__ Summary build_list(uint32_t* hist, int nbins, const int64_t* ov, int oc, int64_t* lv,
                              uint32_t* lc, int lane, const double* __restrict__ ln, int64_t n,
                              bool want_fp) {
  const uint64_t below = lanes_below(lane);
  const bool packed = n < ((int64_t)1 << 21);
  U128 S = {0, 0};
  uint64_t fp = 0;
  int64_t xmax = 0;
  int len = 0;
  // 1. non-zero histogram bins, four per lane per step (16-byte LDS reads;
  //    nbins is a multiple of 256), compacted in ascending order.  A bin's
  //    list position never exceeds its own index, so the packed copy only
  //    overwrites bins that have been read.
  for (int b0 = 0; b0 < nbins; b0 += 256) {
    const uint4 h = *reinterpret_cast<const uint4*>(hist + b0 + 4 * lane);
    const uint32_t nz = (h.x != 0u) + (h.y != 0u) + (h.z != 0u) + (h.w != 0u);
    const uint64_t m0 = __ballot(nz & 1u), m1 = __ballot(nz & 2u), m2 = __ballot(nz & 4u);
    int pos = len + __popcll(m0 & below) + 2 * __popcll(m1 & below) + 4 * __popcll(m2 & below);
    const uint32_t v0 = (uint32_t)(b0 + 4 * lane + 1);
    const uint32_t cs[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (cs[k]) {
        lv[pos] = (int64_t)(v0 + k);
        lc[pos] = cs[k];
        if (packed) hist[pos] = ((v0 + k) << 21) | cs[k];
        ++pos;
      }
    }
    len += __popcll(m0) + 2 * __popcll(m1) + 4 * __popcll(m2);
  }
  const int hlen = len;
  // 2. runs of equal values in the sorted overflow array; the last lane of a
  //    run adds the run's terms.  A run starts at the last start position at
  //    or below its end: in this chunk (ballot of starts), else the carried
  //    start of a run that began in an earlier chunk.
  int run0 = 0;  // start of the run open at the chunk boundary (wave-uniform)
  for (int p0 = 0; p0 < oc; p0 += 64) {
    const int p = p0 + lane;
    const bool valid = p < oc;
    const int64_t v = valid ? ov[p] : 0;
    // neighbours read at clamped indices (always inside ov[0..oc))
    const int64_t vn = ov[p + 1 < oc ? p + 1 : oc - 1];
    const int64_t vp = ov[p > 0 ? (p - 1 < oc ? p - 1 : oc - 1) : 0];
    const bool end = valid && ((p == oc - 1) || (vn != v));
    const bool start = valid && ((p == 0) || (vp != v));
    const uint64_t m = __ballot(end);
    const uint64_t sm = __ballot(start);
    if (end) {
      const int pos = len + __popcll(m & below);
      const uint64_t sb = sm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
      const int first = sb ? p0 + 63 - __clzll((long long)sb) : run0;
      const uint32_t cnt = (uint32_t)(p + 1 - first);
      lv[pos] = v;
      lc[pos] = cnt;
      u128_add_mul(S, cnt, ln_fixed(v, ln));
      if (want_fp) {
        fp += (uint64_t)cnt * mix64((uint64_t)v);
        xmax = v > xmax ? v : xmax;
      }
    }
    len += __popcll(m);
    if (sm) run0 = p0 + 63 - __clzll((long long)sm);
  }
  // 3. exact S (and fingerprint, max) over the histogram part of the list
  if (packed) {
    wave_sync();
    for (int q = lane; q < hlen; q += 64) {
      const uint32_t e = hist[q];
      const int64_t v = (int64_t)(e >> 21);
      const uint32_t c = e & ((1u << 21) - 1u);
      u128_add_mul(S, c, ln_fixed(v, ln));
      if (want_fp) {
        fp += (uint64_t)c * mix64((uint64_t)v);
        xmax = v > xmax ? v : xmax;
      }
    }
  } else {
    wave_sync_global();  // the list is in global memory
    for (int q = lane; q < hlen; q += 64) {
      const int64_t v = lv[q];
      const uint32_t c = lc[q];
      u128_add_mul(S, c, ln_fixed(v, ln));
      if (want_fp) {
        fp += (uint64_t)c * mix64((uint64_t)v);
        xmax = v > xmax ? v : xmax;
      }
    }
  }
  Summary s;
  s.S = wave_sum_u128(S);
  s.fp = want_fp ? wave_sum_u64(fp) : 0ull;
  s.xmax = want_fp ? wave_max_i64(xmax) : 0;
  s.len = len;
  return s;
}

// Ascending sort of up to 64 values held one per lane (unused lanes hold
// INT64_MAX): a bitonic network over lane shuffles, no memory traffic.
__device__ __forceinline__ int64_t wave_sort64(int64_t v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int64_t o = (int64_t)shfl_xor_u64((uint64_t)v, j);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const int64_t lo = o < v ? o : v, hi = o < v ? v : o;
      v = (lower == up) ? lo : hi;
    }
  }
  return v;
}

__device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Compare-exchange of a (the lower index) and b: the smaller value goes to a
// when the block holding them sorts ascending (up), the larger otherwise.
__device__ __forceinline__ void cmpx(int64_t& a, int64_t& b, bool up) {
  const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = up ? lo : hi;
  b = up ? hi : lo;
}

// Passes j = jtop..1 of bitonic stage k on a block of 64 E elements held E
// per lane: element t of this lane has index base + lane + 64 t.  Passes with
// j >= 64 pair registers t and t | j/64 of the same lane; passes with j < 64
// pair lanes (shuffles).  Every index is a compile-time register number.
template <int E>
__device__ __forceinline__ void block_passes(int64_t (&v)[E], int base, int k, int jtop,
                                             int lane) {
#pragma unroll
  for (int tj = E / 2; tj >= 1; tj >>= 1) {
    if ((tj << 6) <= jtop) {
#pragma unroll
      for (int t = 0; t < E; ++t)
        if ((t & tj) == 0) cmpx(v[t], v[t | tj], ((base + lane + 64 * t) & k) == 0);
    }
  }
#pragma unroll
  for (int j = 32; j > 0; j >>= 1) {
    if (j <= jtop) {
      const bool lower = (lane & j) == 0;
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const bool up = ((base + lane + 64 * t) & k) == 0;
        const int64_t o = (int64_t)shfl_xor_u64((uint64_t)v[t], j);
        const int64_t lo = o < v[t] ? o : v[t], hi = o < v[t] ? v[t] : o;
        v[t] = (lower == up) ? lo : hi;
      }
    }
  }
}

// Every stage k <= 64 E of a block (a full bitonic sort when the block is the
// whole array; else a sort whose direction alternates with the block index,
// as the network's first stages leave it).
template <int E>
__device__ __forceinline__ void block_sort(int64_t (&v)[E], int base, int lane) {
  for (int k = 2; k <= 64 * E; k <<= 1) block_passes<E>(v, base, k, k >> 1, lane);
}

template <int E>
__device__ __forceinline__ void block_load(int64_t (&v)[E], const int64_t* a, int lane) {
#pragma unroll
  for (int t = 0; t < E; ++t) v[t] = a[lane + 64 * t];
}
template <int E>
__device__ __forceinline__ void block_store(const int64_t (&v)[E], int64_t* a, int lane) {
#pragma unroll
  for (int t = 0; t < E; ++t) a[lane + 64 * t] = v[t];
}

// Ascending bitonic sort of a[0..P) (P a power of two, 128..512) by one wave,
// entirely in registers (P / 64 values per lane); a is LDS or global memory,
// read once and written once by the calling wave.
__device__ __forceinline__ void wave_sort_small(int64_t* a, int P, int lane) {
  if (P == 128) {
    int64_t v[2];
    block_load<2>(v, a, lane);
    block_sort<2>(v, 0, lane);
    block_store<2>(v, a, lane);
  } else if (P == 256) {
    int64_t v[4];
    block_load<4>(v, a, lane);
    block_sort<4>(v, 0, lane);
    block_store<4>(v, a, lane);
  } else {
    int64_t v[8];
    block_load<8>(v, a, lane);
    block_sort<8>(v, 0, lane);
    block_store<8>(v, a, lane);
  }
}

// The same for a[0..nv) padded to P: positions from nv on count as INT64_MAX
// and are neither read nor written (the wave form's LDS area holds fewer
// than P entries).
template <int E>
__device__ __forceinline__ void block_load_n(int64_t (&v)[E], const int64_t* a, int nv, int lane) {
#pragma unroll
  for (int t = 0; t < E; ++t) v[t] = lane + 64 * t < nv ? a[lane + 64 * t] : INT64_MAX;
}
template <int E>
__device__ __forceinline__ void block_store_n(const int64_t (&v)[E], int64_t* a, int nv, int lane) {
#pragma unroll
  for (int t = 0; t < E; ++t)
    if (lane + 64 * t < nv) a[lane + 64 * t] = v[t];
}
__device__ __forceinline__ void wave_sort_small_n(int64_t* a, int P, int nv, int lane) {
  if (P == 128) {
    int64_t v[2];
    block_load_n<2>(v, a, nv, lane);
    block_sort<2>(v, 0, lane);
    block_store_n<2>(v, a, nv, lane);
  } else {
    int64_t v[4];
    block_load_n<4>(v, a, nv, lane);
    block_sort<4>(v, 0, lane);
    block_store_n<4>(v, a, nv, lane);
  }
}

// G consecutive passes j1, j1/2, ..., j1 >> (G-1) (all >= 512) of bitonic
// stage k over g[0..P) in one round trip: each group of 2^G elements differing
// only in those index bits is loaded into registers, put through the G passes
// and stored back.  The block direction (index & k) is the same for a whole
// group, since k is above every bit that varies in it.
template <int G>
__device__ __forceinline__ void mem_group(int64_t* g, int P, int k, int j1, int lane) {
  constexpr int NE = 1 << G;
  const int p = 31 - __builtin_clz((unsigned)j1);
  const int low = p - G + 1;
  const int lowmask = (1 << low) - 1;
  // two groups per lane per step (P >> G is a multiple of 128 for P >= 1024),
  // all their loads in flight before the compare-exchanges
  for (int q = lane; q < (P >> G); q += 128) {
    int b[2];
    int64_t v[2][NE];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int qq = q + 64 * h;
      b[h] = ((qq >> low) << (p + 1)) | (qq & lowmask);
#pragma unroll
      for (int e = 0; e < NE; ++e) v[h][e] = g[b[h] + (e << low)];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool up = (b[h] & k) == 0;
#pragma unroll
      for (int sft = G - 1; sft >= 0; --sft) {
#pragma unroll
        for (int e = 0; e < NE; ++e)
          if ((e & (1 << sft)) == 0) cmpx(v[h][e], v[h][e | (1 << sft)], up);
      }
#pragma unroll
      for (int e = 0; e < NE; ++e) g[b[h] + (e << low)] = v[h][e];
    }
  }
}

// Ascending bitonic sort of the global array g[0..P) (P a power of two, at
// least 128) by one wave.  Arrays of up to 512 values are sorted in registers.
// Larger ones: every 512-value block is first sorted in registers (the
// network's stages up to 512); each later stage k runs its passes with
// j >= 512 through memory, up to three per round trip (mem_group), and its
// passes with j <= 256 on 512-value blocks in registers.  A 4,096-value
// array takes 7 round trips through memory instead of 78 passes.
__device__ void wave_sort_global(int64_t* g, int P, int lane) {
  if (P <= 512) {
    wave_sort_small(g, P, lane);
    wave_sync_global();
    return;
  }
  // two 512-value blocks per step (P >= 1024 holds an even number), both
  // blocks' loads in flight together
  for (int base = 0; base < P; base += 1024) {
    int64_t v[8], w[8];
    block_load<8>(v, g + base, lane);
    block_load<8>(w, g + base + 512, lane);
    block_sort<8>(v, base, lane);
    block_sort<8>(w, base + 512, lane);
    block_store<8>(v, g + base, lane);
    block_store<8>(w, g + base + 512, lane);
  }
  wave_sync_global();
  for (int k = 1024; k <= P; k <<= 1) {
    int j = k >> 1;
    while (j >= 512) {
      const int G = min(3, 31 - __builtin_clz((unsigned)j) - 8);
      if (G == 3)
        mem_group<3>(g, P, k, j, lane);
      else if (G == 2)
        mem_group<2>(g, P, k, j, lane);
      else
        mem_group<1>(g, P, k, j, lane);
      wave_sync_global();
      j >>= G;
    }
    for (int base = 0; base < P; base += 1024) {
      int64_t v[8], w[8];
      block_load<8>(v, g + base, lane);
      block_load<8>(w, g + base + 512, lane);
      block_passes<8>(v, base, k, 256, lane);
      block_passes<8>(w, base + 512, k, 256, lane);
      block_store<8>(v, g + base, lane);
      block_store<8>(w, g + base + 512, lane);
    }
    wave_sync_global();
  }
}

__device__ __forceinline__ int64_t resolve_entry(uint64_t e, uint32_t rep, const DevCell& c,
                                                 const uint64_t* __restrict__ T,
                                                 const uint32_t* __restrict__ guide,
                                                 uint32_t& fl) {
  if (e >> 63)
    return tail_draw(c.beta, c.gm, c.k0, c.k1, (uint32_t)e, rep, c.stream, &fl);  // inline: no call in the draw loop
  return (int64_t)slow_search(e & ((1ull << 53) - 1), T, guide, (int)c.gsh);
}

// Ring of deferred draws (lane and wave forms).  Before an iteration's
// appends (at most 64 lanes x 4 draws) it holds fewer than 64 entries, so
// 320 entries never overflow.
constexpr int kRing = 320;

// Appends the draws d with def[d] set (at most 4 per lane) to the ring at
// head qh holding qn entries; qn is wave-uniform.  Positions come from a
// wave prefix sum of the per-lane counts (three ballots of its bits).
template <int ND, class Entry>
__device__ __forceinline__ void ring_append(uint64_t* ring, uint32_t qh, uint32_t& qn,
                                            const bool (&def)[ND], Entry entry, int lane) {
  static_assert(ND <= 4, "per-lane count must fit in 3 bits");
  uint32_t nd = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) nd += def[d] ? 1u : 0u;
  if (__ballot(nd != 0u) == 0ull) return;
  const uint64_t below = lanes_below(lane);
  const uint64_t m0 = __ballot(nd & 1u), m1 = __ballot(nd & 2u), m2 = __ballot(nd & 4u);
  uint32_t pos = qh + qn + (uint32_t)(__popcll(m0 & below) + 2 * __popcll(m1 & below) +
                                      4 * __popcll(m2 & below));
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (def[d]) {
      ring[pos >= (uint32_t)kRing ? pos - (uint32_t)kRing : pos] = entry(d);
      ++pos;
    }
  }
  qn += (uint32_t)(__popcll(m0) + 2 * __popcll(m1) + 4 * __popcll(m2));
}

// ---------------------------------------------------------------------------
// LDS of the simulation kernel: the cell's CDF table and packed guide, and one
// region per wave (lane form or wave form).
// ---------------------------------------------------------------------------
static_assert(kHLB % 2 == 0, "two 16-bit counters per dword; value kHLB + 1 maps to the pad row");
static_assert(64 * 2 * kLaneCap <= kListCap,
              "the lane form's value slots and sorted lists fit the wave's list scratch");
struct alignas(16) LaneRegion {
  // dword b of lane l at hist[b * 64 + l]; row kHLB / 2 is a pad that takes
  // the draw loop's no-op counts (never read)
  uint32_t hist[(kHLB / 2 + 1) * 64];
  uint64_t ring[kRing];          // deferred draws
  uint32_t ovc[64];  // values the drains added to a lane's list (may exceed its room)
  uint32_t fl[64];   // flags per lane
};

// Wave-form histogram layout: bins of values 1..kHW, one pad slot per lane
// (the draw loop's no-op counts, never read), then three rows of per-lane
// counts of the values 1, 2 and 3 (most draws: a lane counting into its own
// slot never conflicts with another lane).
constexpr int kWavePad = kHW;
constexpr int kWaveOwn = kHW + 64;
struct alignas(16) WaveRegion {
  uint32_t hist[kHW + 64 + 3 * 64];
  int64_t ov[kCW];
  uint64_t ring[kRing];     // deferred draws
  uint32_t ovc;
};

union WaveLds {
  LaneRegion lane;
  WaveRegion wave;
};

struct SimLds {
  alignas(16) uint64_t T[kH];  // floor(F(k) 2^53)
  uint32_t guide[kGuide];
  WaveLds w[kWaves];
  int unit;
};
static_assert(sizeof(SimLds) <= 160 * 1024, "the simulation kernel's LDS fits one compute unit");

// Out of line: inlined into the persistent kernels' cell switch it takes
// registers from their hot loops.
static __device__ __noinline__ uint32_t guide_pack_dev(const uint16_t* g, int b, int sh,
                                                       uint64_t timax) {
  return guide_pack(g, b, sh, timax);
}

// Stages the cell's table, as integers floor(F(k) 2^53), and packed guide
// (guide_pack) into LDS.
__device__ __forceinline__ void load_cell_tables(uint64_t* T, uint32_t* guide,
                                                 const double* __restrict__ Tg,
                                                 const uint16_t* __restrict__ g,
                                                 const DevCell& c, int tid, int nthreads) {
  for (int k = tid; k < kH; k += nthreads) T[k] = table_int(Tg[k]);
  const uint64_t timax = table_int(c.tmax);
  const int sh = (int)c.gsh;
  for (int b = tid; b < kGuide; b += nthreads) guide[b] = guide_pack_dev(g, b, sh, timax);
}

// ---------------------------------------------------------------------------
// Lane form: one replicate per lane.  Fast-path draws go straight into the
// lane's histogram column; deferred draws from all lanes are resolved 64 at a
// time by whichever lane picks them up, into the owner's column.
// ---------------------------------------------------------------------------
// The lane's larger values take kLaneCap slots of the wave's global scratch,
// slot s of lane l at spill[s * 64 + l].  The lane's own draws fill slots
// 0, 1, ... (a register count); the drains, which resolve any lane's draws,
// fill slots kLaneCap - 1, kLaneCap - 2, ... (an LDS count per owner).
__device__ __forceinline__ void lane_slot_store(LaneRegion* L, int64_t* spill, int owner, int s,
                                                int64_t x) {
  spill[s * 64 + owner] = x;
}
__device__ __forceinline__ void lane_insert(LaneRegion* L, int64_t* spill, int owner, int64_t x) {
  if (x <= kHLB) {
    const int v = (int)x - 1;
    atomicAdd(&L->hist[(v >> 1) * 64 + owner], 1u << ((v & 1) * 16));
  } else {
    const uint32_t p = atomicAdd(&L->ovc[owner], 1u);
    if (p < (uint32_t)kLaneCap) lane_slot_store(L, spill, owner, kLaneCap - 1 - (int)p, x);
  }
}

// Resolves ring entries [qh, qh + m) (one per lane) into the owners'
// columns.  The leading wave_sync makes entries written by other lanes
// visible; every caller is in wave-uniform control flow.
__device__ __forceinline__ void lane_drain(LaneRegion* L, int64_t* spill, int m, uint32_t qh,
                                           int64_t rep0, const DevCell& c,
                                           const uint64_t* __restrict__ T,
                                           const uint32_t* __restrict__ guide, int lane) {
  wave_sync();
  if (lane < m) {
    uint32_t p = qh + (uint32_t)lane;
    if (p >= (uint32_t)kRing) p -= (uint32_t)kRing;
    const uint64_t e = L->ring[p];
    const int owner = (int)((e >> 53) & 63u);
    uint32_t fl = 0;
    const int64_t x = resolve_entry(e, (uint32_t)(rep0 + owner), c, T, guide, fl);
    if (fl) atomicOr(&L->fl[owner], fl);
    lane_insert(L, spill, owner, x);
  }
}

// Draw blocks per iteration of the lane form's loop (two draws each).
constexpr int kLaneBlocks = 2;  // four draws per lane and iteration
static_assert(kLaneBlocks == 2, "the draw loop keeps four table reads in flight");

__device__ __forceinline__ void lane_wave(const DevCell& c, int32_t cell_id, int64_t rep0,
                                          int count, LaneRegion* L, int lane,
                                          const uint64_t* __restrict__ T,
                                          const uint32_t* __restrict__ guide,
                                          const double* __restrict__ ln, const Outputs& out,
                                          uint64_t* esc_list, uint32_t* esc_count,
                                          uint32_t esc_cap, uint32_t* err, int64_t* spill) {
  const bool active = lane < count;
#pragma unroll
  for (int b = 0; b < kHLB / 2; ++b) L->hist[b * 64 + lane] = 0u;
  L->ovc[lane] = 0u;
  L->fl[lane] = 0u;
  wave_sync();
  const int64_t n = c.n;
  const uint32_t r = (uint32_t)(rep0 + lane);
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  // Deferred draws wait in a ring (head qh, qn entries, both wave-uniform).
  uint32_t qh = 0, qn = 0;
  int myc = 0;  // the lane's own values above the column
  const uint64_t timax = table_int(c.tmax);
  const int sh = (int)c.gsh;
  const uint32_t n32 = (uint32_t)n;  // draw indexes are 32-bit
  // The loop is software-pipelined: an iteration issues the guide reads of
  // its uniforms, generates the next iteration's uniforms while they are in
  // flight, issues the table reads, and computes the next guide indexes while
  // those are in flight (one extra block of uniforms is generated at the end).
  auto gen = [&](uint32_t j, uint64_t (&Uo)[2 * kLaneBlocks]) {
    // the round keys are recomputed per block with scalar adds rather than
    // kept live across the loop (where they would be spilled)
    uint32_t k0 = c.k0, k1 = c.k1;
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int b = 0; b < kLaneBlocks; ++b) {
      const Words4 w = philox4x32_10(j + (uint32_t)b, r, c.stream, 0u, k0, k1);
      Uo[2 * b] = m53(w.w0, w.w1);
      Uo[2 * b + 1] = m53(w.w2, w.w3);
    }
  };
  uint64_t U[2 * kLaneBlocks];  // uniforms as 53-bit integers m
  int gi[2 * kLaneBlocks];      // their guide bins
  gen(0u, U);
#pragma unroll
  for (int d = 0; d < 2 * kLaneBlocks; ++d) gi[d] = guide_index(U[d], sh);
  for (uint32_t j = 0; j < nblk; j += kLaneBlocks) {
    uint32_t gg[2 * kLaneBlocks];
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) gg[d] = guide[gi[d]];
    uint64_t Un[2 * kLaneBlocks];
    gen(j + (uint32_t)kLaneBlocks, Un);
    asm volatile("" : "+v"(Un[0]), "+v"(Un[1]), "+v"(Un[2]), "+v"(Un[3]));  // made here
    uint64_t t[2 * kLaneBlocks];
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) t[d] = T[(int)(gg[d] & 0xffffu) - 1];
    __builtin_amdgcn_sched_barrier(0);  // the table reads issue before the index math
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) gi[d] = guide_index(Un[d], sh);
    asm volatile("" : "+v"(gi[0]), "+v"(gi[1]), "+v"(gi[2]), "+v"(gi[3]));  // made here
    asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]));  // reads stay unconditional
    int x[2 * kLaneBlocks];
    bool def[2 * kLaneBlocks];
    bool big = false;
    int xf[2 * kLaneBlocks];
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) xf[d] = fast_select(gg[d], t[d], U[d]);
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) {
      const bool valid = active && 2u * j + (uint32_t)d < n32;
      const int xd = xf[d];
      const bool drawn = xd < kDeferred;
      x[d] = valid && drawn ? xd : -1;
      def[d] = valid && !drawn;
      big = big || x[d] > kHLB;
      // own column, no branch: values outside 1..kHLB count into the pad row
      const uint32_t xm1 = (uint32_t)(x[d] - 1);
      const uint32_t v = xm1 < (uint32_t)kHLB ? xm1 : (uint32_t)kHLB;
      atomicAdd(&L->hist[(v >> 1) * 64 + lane], 1u << ((v & 1u) * 16u));
    }
    if (__ballot(big) != 0ull) {  // values above the column, into the lane's own slots
#pragma unroll
      for (int d = 0; d < 2 * kLaneBlocks; ++d) {
        if (x[d] > kHLB) {
          if (myc < kLaneCap) lane_slot_store(L, spill, lane, myc, x[d]);
          ++myc;
        }
      }
    }
    ring_append(L->ring, qh, qn, def, [&](int d) {
      return defer_entry(U[d], timax, 2u * j + (uint32_t)d, lane);
    }, lane);
    while (qn >= 64u) {
      lane_drain(L, spill, 64, qh, rep0, c, T, guide, lane);
      qh = qh + 64u >= (uint32_t)kRing ? qh + 64u - (uint32_t)kRing : qh + 64u;
      qn -= 64u;
    }
#pragma unroll
    for (int d = 0; d < 2 * kLaneBlocks; ++d) U[d] = Un[d];
  }
  if (qn > 0u) lane_drain(L, spill, (int)qn, qh, rep0, c, T, guide, lane);
  wave_sync_global();  // other lanes' drains wrote to this lane's spill entries
  if (!active) return;
  const int od = (int)L->ovc[lane];
  const int oc = myc + od;
  const uint32_t fl = L->fl[lane];
  if (oc > kLaneCap) {
    const uint32_t slot = atomicAdd(esc_count, 1u);
    if (slot < esc_cap)
      esc_list[slot] = ((uint64_t)(uint32_t)cell_id << 32) | r;
    else
      atomicOr(err, kErrEscOverflow);
    return;
  }
  uint32_t* h = L->hist + lane;
  U128 S = {0, 0};
  uint64_t fp = 0;
  int64_t xmax = 0;
  // The larger values sorted into the scratch after the spill area: each
  // goes to its rank (values below it, plus equal ones stored before it; no
  // data-dependent moves), eight values at a time against one pass over all
  // of them (independent reads), and the order-free sums are taken on the way.
  // Value q of the lane: its own slots 0..myc-1, then the drains' slots.
  const int64_t* g = spill + lane;
  int64_t* srt = spill + 64 * kLaneCap + lane;  // entry p at srt[p * 64]
  auto ovv = [&](int q) -> int64_t {
    return g[(q < myc ? q : kLaneCap - od + (q - myc)) * 64];
  };
  for (int i0 = 0; i0 < oc; i0 += 8) {
    int64_t v[8];
    int rank[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      v[t] = i0 + t < oc ? ovv(i0 + t) : INT64_MAX;
      rank[t] = 0;
    }
#pragma unroll 4
    for (int j = 0; j < oc; ++j) {
      const int64_t w = ovv(j);
#pragma unroll
      for (int t = 0; t < 8; ++t) rank[t] += (w < v[t] || (w == v[t] && j < i0 + t)) ? 1 : 0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (i0 + t < oc) {
        srt[rank[t] * 64] = v[t];
        u128_add(S, ln_fixed(v[t], ln), 0);
        fp += mix64((uint64_t)v[t]);
        xmax = v[t] > xmax ? v[t] : xmax;
      }
    }
  }
  for (int b = 0; b < kHLB / 2; ++b) {
    const uint32_t wv = h[b * 64];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const uint32_t k = half ? (wv >> 16) : (wv & 0xffffu);
      const int64_t v = 2 * b + half + 1;
      if (k) {
        u128_add_mul(S, k, ln_fixed(v, ln));
        fp += (uint64_t)k * mix64((uint64_t)v);
        xmax = v > xmax ? v : xmax;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the sorted list is read back
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  LaneSrc src{h, srt, oc, 17, 0};
  double a, D;
  uint32_t flags;
  finish_replicate(src, S, n, fl, ln, c.K, a, D, flags);
  write_outputs(out, c.out_off + rep0 + lane, D, a, flags, fp, xmax);
}

// ---------------------------------------------------------------------------
// Wave form: one wave draws one replicate at a time into an LDS histogram;
// finishes are deferred and run one replicate per lane.
// ---------------------------------------------------------------------------
struct WaveSlot {
  U128 S;
  uint64_t fp;
  int64_t xmax;
  uint32_t off, len, flags, esc;
};

__device__ __forceinline__ void wave_insert(WaveRegion* L, int64_t x) {
  if (x <= kHW) {
    atomicAdd(&L->hist[x - 1], 1u);
  } else {
    const uint32_t p = atomicAdd(&L->ovc, 1u);
    if (p < (uint32_t)kCW) L->ov[p] = x;
  }
}

// Resolves ring entries [qh, qh + m) (one per lane) into the histogram (see
// lane_drain).
// xm: the lane's largest value counted in the histogram so far.
__device__ __forceinline__ void wave_drain(WaveRegion* L, int m, uint32_t qh, uint32_t rep,
                                           const DevCell& c, const uint64_t* __restrict__ T,
                                           const uint32_t* __restrict__ guide, uint32_t& fl,
                                           int& xm, int lane) {
  wave_sync();
  int64_t v = 0;
  if (lane < m) {
    uint32_t p = qh + (uint32_t)lane;
    if (p >= (uint32_t)kRing) p -= (uint32_t)kRing;
    v = resolve_entry(L->ring[p], rep, c, T, guide, fl);
    wave_insert(L, v);
  }
  xm = max(xm, v <= kHW ? (int)v : 0);
}

// Draw blocks per lane per iteration of the wave form's loop.
constexpr int kWaveBlocks = 2;
static_assert(kWaveBlocks == 2, "the draw loop keeps four table reads in flight");

__device__ __forceinline__ void wave_batch(const DevCell& c, int32_t cell_id, int64_t r0,
                                           int nrep, WaveRegion* L, WaveSlot* slots,
                                           int64_t* __restrict__ lv, uint32_t* __restrict__ lc,
                                           int lane, const uint64_t* __restrict__ T,
                                           const uint32_t* __restrict__ guide,
                                           const double* __restrict__ ln, const Outputs& out,
                                           uint64_t* esc_list, uint32_t* esc_count,
                                           uint32_t esc_cap, uint32_t* err) {
  const int64_t n = c.n;
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  int done = 0;
  // histogram bins [0, hi) may be nonzero: the whole histogram at first (the
  // region's LDS held other data), afterwards the 256-bin blocks up to the
  // previous replicate's largest histogram value (the list build packs its
  // entries below that too)
  int hi = kHW;
  while (done < nrep) {
    // fill a batch of replicates while the list area has room for a worst case
    int q = 0;
    uint32_t used = 0;
    while (done + q < nrep && q < 64 && used + (uint32_t)(kHW + kCW) <= (uint32_t)kListCap) {
      const uint32_t r = (uint32_t)(r0 + done + q);
      for (int k = lane; k < hi; k += 64) L->hist[k] = 0u;
#pragma unroll
      for (int k = 0; k < 3; ++k) L->hist[kWaveOwn + k * 64 + lane] = 0u;
      if (lane == 0) L->ovc = 0u;
      wave_sync();
      int xm = 0;  // the lane's largest table value (clamped to kHW after the loop)
      uint32_t fl = 0;
      uint32_t qh = 0, qn = 0;  // deferred-draw ring, wave-uniform
      const uint64_t timax = table_int(c.tmax);
      const int sh = (int)c.gsh;
      const uint32_t n32 = (uint32_t)n;  // n <= 2^31
      // software-pipelined as the lane form's loop
      auto gen = [&](uint32_t j0, uint64_t (&Uo)[2 * kWaveBlocks]) {
        uint32_t k0 = c.k0, k1 = c.k1;  // round keys per block (see lane_wave)
        asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
        for (int b = 0; b < kWaveBlocks; ++b) {
          const Words4 w = philox4x32_10(j0 + 64u * (uint32_t)b + (uint32_t)lane, r, c.stream,
                                         0u, k0, k1);
          Uo[2 * b] = m53(w.w0, w.w1);
          Uo[2 * b + 1] = m53(w.w2, w.w3);
        }
      };
      uint64_t U[2 * kWaveBlocks];  // uniforms as 53-bit integers m
      int gi[2 * kWaveBlocks];      // their guide bins
      gen(0u, U);
#pragma unroll
      for (int d = 0; d < 2 * kWaveBlocks; ++d) gi[d] = guide_index(U[d], sh);
      for (uint32_t j0 = 0; j0 < nblk; j0 += 64u * kWaveBlocks) {
        uint32_t gg[2 * kWaveBlocks];
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) gg[d] = guide[gi[d]];
        uint64_t Un[2 * kWaveBlocks] = {1ull, 1ull, 1ull, 1ull};
        if (j0 + 64u * kWaveBlocks < nblk) gen(j0 + 64u * kWaveBlocks, Un);  // none past the end
        asm volatile("" : "+v"(Un[0]), "+v"(Un[1]), "+v"(Un[2]), "+v"(Un[3]));  // made here
        uint64_t t[2 * kWaveBlocks];
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) t[d] = T[(int)(gg[d] & 0xffffu) - 1];
        __builtin_amdgcn_sched_barrier(0);  // the table reads issue before the index math
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) gi[d] = guide_index(Un[d], sh);
        asm volatile("" : "+v"(gi[0]), "+v"(gi[1]), "+v"(gi[2]), "+v"(gi[3]));  // made here
        asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]));  // reads stay unconditional
        int x[2 * kWaveBlocks];
        bool def[2 * kWaveBlocks];
        bool big = false;
        int xf[2 * kWaveBlocks];
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) xf[d] = fast_select(gg[d], t[d], U[d]);
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) {
          const uint32_t i = 2u * (j0 + 64u * (uint32_t)(d >> 1) + (uint32_t)lane) + (uint32_t)(d & 1);
          const bool valid = i < n32;
          const int xd = xf[d];
          const bool drawn = xd < kDeferred;
          x[d] = valid && drawn ? xd : -1;
          def[d] = valid && !drawn;
          big = big || x[d] > kHW;
          // 1..3 count into the lane's own row, 4..kHW into their bin, and
          // every other lane adds 1 to its pad slot (no divergent branch)
          const uint32_t xm1 = (uint32_t)(x[d] - 1);
          const int slot = xm1 < 3u ? kWaveOwn + (int)xm1 * 64 + lane
                                    : (xm1 < (uint32_t)kHW ? (int)xm1 : kWavePad + lane);
          atomicAdd(&L->hist[slot], 1u);
          xm = max(xm, x[d]);  // values above kHW are clamped once, below
        }
        if (__ballot(big) != 0ull) {  // values above the histogram
#pragma unroll
          for (int d = 0; d < 2 * kWaveBlocks; ++d)
            if (x[d] > kHW) wave_insert(L, x[d]);
        }
        ring_append(L->ring, qh, qn, def, [&](int d) {
          return defer_entry(U[d], timax,
                             2u * (j0 + 64u * (uint32_t)(d >> 1) + (uint32_t)lane) + (uint32_t)(d & 1),
                             0);
        }, lane);
        while (qn >= 64u) {
          wave_drain(L, 64, qh, r, c, T, guide, fl, xm, lane);
          qh = qh + 64u >= (uint32_t)kRing ? qh + 64u - (uint32_t)kRing : qh + 64u;
          qn -= 64u;
        }
#pragma unroll
        for (int d = 0; d < 2 * kWaveBlocks; ++d) U[d] = Un[d];
      }
      if (qn > 0u) wave_drain(L, (int)qn, qh, r, c, T, guide, fl, xm, lane);
      fl = wave_or_u32(fl);
      // bins the list build reads: whole 256-bin blocks up to the largest
      // histogram value (every lane's xm is defined: set in converged code)
      hi = ((int)min(wave_max_i64((int64_t)xm), (int64_t)kHW) + 255) & ~255;
      hi = hi < 256 ? 256 : hi;
      wave_sync();
      // the own rows' totals, read and summed in converged code
      const uint32_t c1 = wave_sum_u32(L->hist[kWaveOwn + lane]);
      const uint32_t c2 = wave_sum_u32(L->hist[kWaveOwn + 64 + lane]);
      const uint32_t c3 = wave_sum_u32(L->hist[kWaveOwn + 128 + lane]);
      if (lane == 0) {
        L->hist[0] += c1;  // drains count 1..3 into the bins themselves
        L->hist[1] += c2;
        L->hist[2] += c3;
      }
      wave_sync();
      const uint32_t oc = L->ovc;
      if (oc > (uint32_t)kCW) {
        if (lane == 0) {
          const uint32_t slot = atomicAdd(esc_count, 1u);
          if (slot < esc_cap)
            esc_list[slot] = ((uint64_t)(uint32_t)cell_id << 32) | r;
          else
            atomicOr(err, kErrEscOverflow);
          slots[q].esc = 1u;
        }
        wave_sync();
        ++q;
        continue;
      }
      if (oc > 1 && oc <= 64u) {
        const int64_t v = wave_sort64(lane < (int)oc ? L->ov[lane] : INT64_MAX, lane);
        if (lane < (int)oc) L->ov[lane] = v;
        wave_sync();
      } else if (oc > 64u) {
        const int P = next_pow2((int)oc);
        static_assert(kCW <= 256, "the wave form's overflow is sorted in registers");
        wave_sort_small_n(L->ov, P, (int)oc, lane);  // one LDS read and one write per value
        wave_sync();
      }
      Summary s;
      [[clang::always_inline]] s = build_list(L->hist, hi, L->ov, (int)oc, lv + used, lc + used,
                                              lane, ln, n, out.fp != nullptr || out.xmax != nullptr);
      if (lane == 0) {
        WaveSlot sl;
        sl.S = s.S;
        sl.fp = s.fp;
        sl.xmax = s.xmax;
        sl.off = used;
        sl.len = (uint32_t)s.len;
        sl.flags = fl;
        sl.esc = 0u;
        slots[q] = sl;
      }
      used += (uint32_t)s.len;
      ++q;
    }
    // the batch's lists and slots (global stores by various lanes) become
    // visible to every lane once, here, before the finishes read them; each
    // replicate wrote disjoint positions, so no ordering is needed earlier
    wave_sync_global();
    // deferred finishes, one replicate per lane
    if (lane < q) {
      const WaveSlot sl = slots[lane];
      if (!sl.esc) {
        ListSrc src(lv + sl.off, lc + sl.off, (int)sl.len);
        double a, D;
        uint32_t flags;
        finish_replicate(src, sl.S, n, sl.flags, ln, c.K, a, D, flags);
        write_outputs(out, c.out_off + r0 + done + lane, D, a, flags, sl.fp, sl.xmax);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    wave_sync();
    done += q;
  }
}

// ---------------------------------------------------------------------------
// Persistent simulation kernel: workgroups pull units (a cell and up to 512
// replicates) from a global queue; the cell's table and guide are staged in
// LDS when the cell changes.  Lane-form units give one replicate to each
// lane; wave-form units give 64 replicates to each wave.
// ---------------------------------------------------------------------------
// Three waves per SIMD: the twelve waves' LDS regions and the shared table
// fit one workgroup per compute unit, and the register budget is 168 per lane.
static_assert(kBlock == 768, "twelve waves per workgroup, one workgroup per compute unit");
__global__ __launch_bounds__(kBlock, 3) void k_simulate(
    const DevCell* __restrict__ cells, const double* __restrict__ tables,
    const uint16_t* __restrict__ guides, const double* __restrict__ ln,
    const Unit* __restrict__ units, int n_units, uint32_t* queue, Outputs out,
    uint64_t* esc_list, uint32_t* esc_count, uint32_t esc_cap, int64_t* list_v,
    uint32_t* list_c, WaveSlot* wslots, uint32_t* err) {
  __shared__ SimLds L;
  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t gwave = (int64_t)blockIdx.x * kWaves + wave;
  int64_t* lv = list_v + gwave * kListCap;
  uint32_t* lc = list_c + gwave * kListCap;
  WaveSlot* slots = wslots + gwave * 64;
  int loaded = -1;

  for (;;) {
    if (tid == 0) L.unit = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int u = L.unit;
    if (u >= n_units) break;
    const Unit un = units[u];
    const DevCell c = cells[un.cell];
    if (un.cell != loaded) {
      load_cell_tables(L.T, L.guide, tables + (size_t)un.cell * kH,
                       guides + (size_t)un.cell * (kGuide + 1), c, tid, kBlock);
      loaded = un.cell;
      __syncthreads();
    }
    const int first = wave * 64;
    if (first < un.count) {
      const int nrep = (un.count - first) < 64 ? (un.count - first) : 64;
      if (c.mode == kModeLane)
        lane_wave(c, un.cell, un.r0 + first, nrep, &L.w[wave].lane, lane, L.T, L.guide, ln, out,
                  esc_list, esc_count, esc_cap, err, lv);
      else
        wave_batch(c, un.cell, un.r0 + first, nrep, &L.w[wave].wave, slots, lv, lc, lane, L.T,
                   L.guide, ln, out, esc_list, esc_count, esc_cap, err);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Heavy form: 4 waves per workgroup share the table and guide; each wave
// draws one replicate at a time, keeps values above kHeavyHist in its global
// scratch and sorts them there.  Runs the planned heavy units, then every
// replicate that overflowed the lane or wave form.
// ---------------------------------------------------------------------------
struct alignas(16) HeavyWave {
  uint32_t hist[kHeavyHist + 64];  // values 1..kHeavyHist; then one no-op pad slot per lane
  uint64_t ring[kRing];            // deferred draws (simulated replicates)
  uint32_t ones[64];  // per-lane count of values equal to 1 (the most frequent value)
  uint32_t ovc;
};

struct HeavyLds {
  uint64_t T[kH];  // floor(F(k) 2^53)
  uint32_t guide[kGuide];
  HeavyWave w[kHeavyWaves];
  int item;
};
static_assert(2 * sizeof(HeavyLds) <= 160 * 1024, "two heavy workgroups per compute unit");

struct GlobalSync {
  __device__ void operator()() const { wave_sync_global(); }
};

// Histogram/overflow fill, sort, compact list and finish of one replicate by
// one wave.  fill(sink, flags) calls sink(x) for every value.
// K = 0: the pure law; K > 0: the truncated law on 1..K (values above K are
// invalid, like values below 1).  kInlineList: the list build is inlined (the
// fit kernels; out of line, with the histogram reached through a flat
// pointer, a fit has been seen to return a wrong estimate); else the
// compiler decides (the heavy kernel keeps it out of line, which spares its
// registers, and passes every test).
template <bool kInlineList, class Fill>
__device__ void heavy_core(HeavyWave* W, int64_t n, Fill fill, int64_t* gov, int64_t* lv,
                           uint32_t* lc, const double* __restrict__ ln, uint32_t K, bool want_fp,
                           double& a, double& D, uint32_t& flags, uint64_t& fp, int64_t& xmax,
                           bool& ok, int64_t xmin = 1) {
  const int lane = lane_id();
  for (int k = lane; k < kHeavyHist; k += 64) W->hist[k] = 0u;
  W->ones[lane] = 0u;
  if (lane == 0) W->ovc = 0u;
  wave_sync_global();
  uint32_t fl = 0;
  bool bad = false;
  const int64_t xhi = K ? (int64_t)K : INT64_MAX;
  // sink runs in divergent code (partial draw blocks, deferred draws): the
  // ones go to the lane's own LDS counter (no contention on bin 1), summed
  // from LDS once every lane is back
  auto sink = [&](int64_t x) {
    if (x < 1 || x > xhi) {
      bad = true;
    } else if (x == 1) {
      atomicAdd(&W->ones[lane], 1u);
    } else if (x <= kHeavyHist) {
      atomicAdd(&W->hist[x - 1], 1u);
    } else {
      const uint32_t idx = atomicAdd(&W->ovc, 1u);
      gov[idx] = x;
    }
  };
  fill(sink, fl);
  wave_sync();
  const uint32_t c1 = wave_sum_u32(W->ones[lane]);
  fl = wave_or_u32(fl);
  const uint32_t anybad = wave_or_u32(bad ? 1u : 0u);
  if (lane == 0) W->hist[0] += c1;
  wave_sync_global();
  ok = (anybad == 0u);
  if (!ok) return;
  const int oc = (int)W->ovc;
  if (oc > 1 && oc <= 64) {
    const int64_t v = wave_sort64(lane < oc ? gov[lane] : INT64_MAX, lane);
    if (lane < oc) gov[lane] = v;
    wave_sync_global();
  } else if (oc > 64) {
    const int P = next_pow2(oc);
    for (int k = oc + lane; k < P; k += 64) gov[k] = INT64_MAX;
    wave_sync_global();
    wave_sort_global(gov, P, lane);
  }
  Summary s;
  if constexpr (kInlineList) {
    [[clang::always_inline]] s = build_list(W->hist, kHeavyHist, gov, oc, lv, lc, lane, ln, n,
                                            want_fp);
  } else {
    s = build_list(W->hist, kHeavyHist, gov, oc, lv, lc, lane, ln, n, want_fp);
  }
  wave_sync_global();
  finish_replicate_wave(lv, lc, s.len, s.S, n, fl, ln, lane, K, a, D, flags, xmin);
  fp = s.fp;
  xmax = s.xmax;
}

// Adds one value per lane (lanes with valid set) to a simulated heavy-form
// replicate, in wave-uniform control flow: ones to the wave's scalar count
// (ballot), 2..kHeavyHist to the LDS histogram (lanes with nothing to add put
// a zero into their own pad slot), larger values to the global overflow array
// at positions from a ballot prefix (no atomics on a shared counter).
__device__ __forceinline__ void heavy_put(HeavyWave* W, int64_t* gov, int64_t v, bool valid,
                                          uint32_t& ones, uint32_t& ovn, int lane,
                                          uint64_t below) {
  ones += (uint32_t)__popcll(__ballot(valid && v == 1));
  const bool hb = valid && v >= 2 && v <= kHeavyHist;
  atomicAdd(&W->hist[hb ? (int)v - 1 : kHeavyHist + lane], 1u);  // pads are never read
  const bool big = valid && v > kHeavyHist;
  const uint64_t mb = __ballot(big);
  if (mb != 0ull) {
    if (big) gov[ovn + (uint32_t)__popcll(mb & below)] = v;
    ovn += (uint32_t)__popcll(mb);
  }
}

// Resolves a deferred draw of a cell with a lower cutoff (xmin = 1 for the
// pure law): the table index j is the value xmin - 1 + j, the tail starts at
// xmin + kH.
__device__ __forceinline__ int64_t resolve_entry_cut(uint64_t e, uint32_t rep, const DevCell& c,
                                                     const uint64_t* __restrict__ T,
                                                     const uint32_t* __restrict__ guide,
                                                     uint32_t& fl) {
  if (e >> 63)  // inline: heavy tails resolve thousands per replicate
    return tail_draw_from((double)(c.xmin + kH), c.beta, c.gm, c.k0, c.k1, (uint32_t)e, rep,
                          c.stream, &fl);
  return (c.xmin - 1) + (int64_t)slow_search(e & ((1ull << 53) - 1), T, guide, (int)c.gsh);
}

// Resolves ring entries [qh, qh + m) (one per lane) into the replicate.
__device__ __forceinline__ void heavy_drain(HeavyWave* W, int64_t* gov, int m, uint32_t qh,
                                            uint32_t rep, const DevCell& c,
                                            const uint64_t* __restrict__ T,
                                            const uint32_t* __restrict__ guide, uint32_t& fl,
                                            uint32_t& ones, uint32_t& ovn, int lane,
                                            uint64_t below) {
  wave_sync();  // entries appended by other lanes
  int64_t v = 0;
  if (lane < m) {
    uint32_t p = qh + (uint32_t)lane;
    if (p >= (uint32_t)kRing) p -= (uint32_t)kRing;
    v = resolve_entry_cut(W->ring[p], rep, c, T, guide, fl);
  }
  heavy_put(W, gov, v, lane < m, ones, ovn, lane, below);
}

// One simulated replicate by one wave: the wave form's draw loop (two Philox
// blocks per lane per iteration, guide lookups in phases, deferred draws in a
// ring resolved 64 at a time) with the values above the LDS histogram in the
// wave's global overflow array; then heavy_core's sort, list and finish.
__device__ void heavy_replicate(HeavyWave* W, const uint64_t* __restrict__ T,
                                const uint32_t* __restrict__ guide, const DevCell& c,
                                uint32_t rep, int64_t* gov, int64_t* lv, uint32_t* lc,
                                const double* __restrict__ ln, const Outputs& out) {
  const int lane = lane_id();
  const int64_t n = c.n;
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  const uint64_t timax = table_int(c.tmax);
  const int64_t off = c.xmin - 1;  // table index j is the value off + j
  auto fill = [&](auto, uint32_t& fl) {
    const uint64_t below = lanes_below(lane);
    uint32_t ones = 0, ovn = 0;  // wave-uniform
    uint32_t qh = 0, qn = 0;     // deferred-draw ring, wave-uniform
    for (uint32_t j0 = 0; j0 < nblk; j0 += 64u * kWaveBlocks) {
      // round keys per block (see lane_wave); the cell is the wave's, so its
      // key is uniform: read from the first lane into scalar registers
      uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c.k0);
      uint32_t k1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c.k1);
      asm volatile("" : "+s"(k0), "+s"(k1));
      uint64_t U[2 * kWaveBlocks];
#pragma unroll
      for (int b = 0; b < kWaveBlocks; ++b) {
        const Words4 w = philox4x32_10(j0 + 64u * (uint32_t)b + (uint32_t)lane, rep, c.stream,
                                       0u, k0, k1);
        U[2 * b] = m53(w.w0, w.w1);
        U[2 * b + 1] = m53(w.w2, w.w3);
      }
      int xf[2 * kWaveBlocks];
      fast_draw4(U, T, guide, (int)c.gsh, xf);
      bool def[2 * kWaveBlocks];
#pragma unroll
      for (int d = 0; d < 2 * kWaveBlocks; ++d) {
        const uint32_t i =
            2u * (j0 + 64u * (uint32_t)(d >> 1) + (uint32_t)lane) + (uint32_t)(d & 1);
        const bool valid = (int64_t)i < n;
        const bool drawn = xf[d] < kDeferred;
        def[d] = valid && !drawn;
        heavy_put(W, gov, off + (int64_t)xf[d], valid && drawn, ones, ovn, lane, below);
      }
      ring_append(W->ring, qh, qn, def, [&](int d) {
        return defer_entry(U[d], timax,
                           2u * (j0 + 64u * (uint32_t)(d >> 1) + (uint32_t)lane) + (uint32_t)(d & 1),
                           0);
      }, lane);
      while (qn >= 64u) {
        heavy_drain(W, gov, 64, qh, rep, c, T, guide, fl, ones, ovn, lane, below);
        qh = qh + 64u >= (uint32_t)kRing ? qh + 64u - (uint32_t)kRing : qh + 64u;
        qn -= 64u;
      }
    }
    if (qn > 0u) heavy_drain(W, gov, (int)qn, qh, rep, c, T, guide, fl, ones, ovn, lane, below);
    if (lane == 0) {
      W->ones[0] = ones;
      W->ovc = ovn;
    }
  };
  double a = 0.0, D = 0.0;
  uint32_t flags = 0;
  uint64_t fp;
  int64_t xmax;
  bool ok;
  heavy_core<false>(W, n, fill, gov, lv, lc, ln, c.K, out.fp != nullptr || out.xmax != nullptr, a, D,
             flags, fp, xmax, ok, c.xmin);
  if (lane == 0) write_outputs(out, c.out_off + rep, D, a, flags, fp, xmax);
  wave_sync_global();
}

// Two waves per SIMD (two workgroups per compute unit, which the LDS allows):
// the register budget is then 256 per lane, against about 310 the compiler
// takes when unbounded (one wave per SIMD); the few values it spills cost far
// less than the halved latency hiding (the heavy form runs 1.6x faster).
__global__ __launch_bounds__(64 * kHeavyWaves, 2) void k_heavy(
    const DevCell* __restrict__ cells, const double* __restrict__ tables,
    const uint16_t* __restrict__ guides, const double* __restrict__ ln,
    const Unit* __restrict__ units, int n_units, const uint64_t* __restrict__ esc_list,
    const uint32_t* __restrict__ esc_count, uint32_t esc_cap, uint32_t* queues,
    Outputs out, int64_t* scratch, int64_t scratch_stride) {
  __shared__ HeavyLds L;
  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int64_t gw = (int64_t)blockIdx.x * kHeavyWaves + wave;
  int64_t* gov = scratch + gw * scratch_stride;
  // list area after the overflow area: values then counts
  const int64_t half = scratch_stride / 2;
  int64_t* lv = gov + half;
  uint32_t* lc = reinterpret_cast<uint32_t*>(lv + half / 2);
  int loaded = -1;
  // planned heavy units: each wave takes every 4th replicate of the unit
  for (;;) {
    if (tid == 0) L.item = (int)atomicAdd(&queues[0], 1u);
    __syncthreads();
    const int u = L.item;
    __syncthreads();
    if (u >= n_units) break;
    const Unit un = units[u];
    const DevCell c = cells[un.cell];
    if (un.cell != loaded) {
      load_cell_tables(L.T, L.guide, tables + (size_t)un.cell * kH,
                       guides + (size_t)un.cell * (kGuide + 1), c, tid, 64 * kHeavyWaves);
      loaded = un.cell;
      __syncthreads();
    }
    for (int k = wave; k < un.count; k += kHeavyWaves)
      heavy_replicate(&L.w[wave], L.T, L.guide, c, (uint32_t)(un.r0 + k), gov, lv, lc, ln, out);
    __syncthreads();
  }
  // replicates that overflowed the lane or wave form (wave 0 of each group)
  const uint32_t ne = *esc_count < esc_cap ? *esc_count : esc_cap;
  for (;;) {
    if (tid == 0) L.item = (int)atomicAdd(&queues[1], 1u);
    __syncthreads();
    const uint32_t e = (uint32_t)L.item;
    __syncthreads();
    if (e >= ne) break;
    const uint64_t code = esc_list[e];
    const int cell = (int)(code >> 32);
    const uint32_t rep = (uint32_t)code;
    const DevCell c = cells[cell];
    if (cell != loaded) {
      load_cell_tables(L.T, L.guide, tables + (size_t)cell * kH,
                       guides + (size_t)cell * (kGuide + 1), c, tid, 64 * kHeavyWaves);
      loaded = cell;
      __syncthreads();
    }
    if (wave == 0) heavy_replicate(&L.w[0], L.T, L.guide, c, rep, gov, lv, lc, ln, out);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Dataset fit: S, alpha_hat and D of caller data x[0..n) (one wave per
// dataset).  Same histogram/list/finish arithmetic as the simulated
// replicates, so identical multisets give bit-identical results.
// ---------------------------------------------------------------------------
// Bitonic sort of buf[0..P) (P a power of two) by the nthreads threads of
// one workgroup; buf is LDS or global memory (a workgroup shares its CU's
// caches, so the barrier orders the passes either way).
__device__ __forceinline__ void block_bitonic(int64_t* buf, int P, int tid, int nthreads) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += nthreads) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int64_t a = buf[i], b = buf[ixj];
          const bool asc = (i & k) == 0;
          if ((a > b) == asc) {
            buf[i] = b;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Fit of one large dataset (eq. 2 and eq. 3) by a whole workgroup: all
// kFitWaves waves fill the LDS histogram (values 1..kHeavyHist) and the
// global overflow list and sort the overflow (in LDS when it fits); wave 0
// then builds the (value, count) list and finishes as k_fit does, so the
// result has k_fit's bits.
constexpr int kFitWaves = 8;
constexpr int kFitSortLds = 4096;
__global__ __launch_bounds__(64 * kFitWaves) void k_fit_block(
    const int64_t* __restrict__ x, int64_t n, const double* __restrict__ ln, int64_t* scratch,
    int64_t scratch_stride, double* ahat_out, double* D_out, uint32_t* flags_out,
    uint32_t* status_out, uint32_t K) {
  __shared__ HeavyWave W;
  __shared__ int64_t sbuf[kFitSortLds];
  __shared__ uint32_t sbad;
  const int tid = (int)threadIdx.x;
  const int nt = (int)blockDim.x;
  const int lane = tid & 63;
  int64_t* gov = scratch;
  const int64_t half = scratch_stride / 2;
  int64_t* lv = gov + half;
  uint32_t* lc = reinterpret_cast<uint32_t*>(lv + half / 2);
  for (int k = tid; k < kHeavyHist; k += nt) W.hist[k] = 0u;
  if (tid == 0) {
    W.ovc = 0u;
    sbad = 0u;
  }
  __syncthreads();
  const int64_t xhi = K ? (int64_t)K : INT64_MAX;
  uint32_t bad = 0u;
  for (int64_t i = tid; i < n; i += nt) {
    const int64_t v = x[i];
    if (v < 1 || v > xhi) {
      bad = 1u;
    } else if (v <= kHeavyHist) {
      atomicAdd(&W.hist[v - 1], 1u);
    } else {
      const uint32_t idx = atomicAdd(&W.ovc, 1u);
      gov[idx] = v;
    }
  }
  if (bad) atomicOr(&sbad, 1u);
  __syncthreads();
  const bool ok = sbad == 0u;
  const int oc = (int)W.ovc;
  if (ok && oc > 1) {
    const int P = next_pow2(oc);
    if (P <= kFitSortLds) {
      for (int k = tid; k < P; k += nt) sbuf[k] = k < oc ? gov[k] : INT64_MAX;
      __syncthreads();
      block_bitonic(sbuf, P, tid, nt);
      for (int k = tid; k < oc; k += nt) gov[k] = sbuf[k];
    } else {
      for (int k = oc + tid; k < P; k += nt) gov[k] = INT64_MAX;
      __syncthreads();
      block_bitonic(gov, P, tid, nt);
    }
    __syncthreads();
  }
  if (tid >= 64) return;
  if (!ok) {
    if (lane == 0) status_out[0] = kErrBadValue;
    return;
  }
  Summary sm;
  [[clang::always_inline]] sm = build_list(W.hist, kHeavyHist, gov, oc, lv, lc, lane, ln, n, false);
  wave_sync_global();
  double a = 0.0, D = 0.0;
  uint32_t flags = 0;
  finish_replicate_wave(lv, lc, sm.len, sm.S, n, 0u, ln, lane, K, a, D, flags);
  if (lane == 0) {
    ahat_out[0] = a;
    D_out[0] = D;
    flags_out[0] = flags;
    status_out[0] = 0u;
  }
}

// The KS-minimising choice of a lower cutoff (the practice the paper cites
// for fitting data): for each candidate xmin one wave fits the values >= xmin
// of the same dataset (the law with cutoff xmin, eq. 2 and eq. 3 with the
// Hurwitz zeta).  A candidate above every value gets D = +inf and status
// kErrNoTail; any value below 1 sets kErrBadValue.
__global__ __launch_bounds__(64) void k_fit_scan(const int64_t* __restrict__ x, int64_t n,
                                                const int64_t* __restrict__ xmins, int n_cand,
                                                const double* __restrict__ ln, int64_t* scratch,
                                                int64_t scratch_stride, double* ahat_out,
                                                double* D_out, int64_t* ntail_out,
                                                uint32_t* flags_out, uint32_t* status_out) {
  __shared__ HeavyWave W;
  int64_t* gov = scratch + (int64_t)blockIdx.x * scratch_stride;
  const int64_t half = scratch_stride / 2;
  int64_t* lv = gov + half;
  uint32_t* lc = reinterpret_cast<uint32_t*>(lv + half / 2);
  const int lane = lane_id();
  for (int cand = (int)blockIdx.x; cand < n_cand; cand += (int)gridDim.x) {
    const int64_t xmin = xmins[cand];
    uint32_t cnt = 0, bad = 0;
    for (int64_t i = lane; i < n; i += 64) {
      const int64_t v = x[i];
      bad |= v < 1 ? 1u : 0u;
      cnt += v >= xmin ? 1u : 0u;
    }
    cnt = wave_sum_u32(cnt);
    bad = wave_or_u32(bad);
    if (bad != 0u || cnt == 0u) {
      if (lane == 0) {
        ahat_out[cand] = 0.0;
        D_out[cand] = __builtin_inf();
        ntail_out[cand] = (int64_t)cnt;
        flags_out[cand] = 0u;
        status_out[cand] = bad != 0u ? kErrBadValue : kErrNoTail;
      }
      continue;
    }
    auto fill = [&](auto sink, uint32_t&) {
      for (int64_t i = lane; i < n; i += 64) {
        const int64_t v = x[i];
        if (v >= xmin) sink(v);
      }
    };
    double a = 0.0, D = 0.0;
    uint32_t flags = 0;
    uint64_t fp;
    int64_t xmax;
    bool ok;
    heavy_core<true>(&W, (int64_t)cnt, fill, gov, lv, lc, ln, 0u, false, a, D, flags, fp, xmax, ok,
               xmin);
    if (lane == 0) {
      ahat_out[cand] = a;
      D_out[cand] = D;
      ntail_out[cand] = (int64_t)cnt;
      flags_out[cand] = flags;
      status_out[cand] = ok ? 0u : kErrBadValue;
    }
    wave_sync_global();
  }
}

__global__ __launch_bounds__(64) void k_fit(const int64_t* const* __restrict__ xs,
                                           const int64_t* __restrict__ ns, int n_sets,
                                           const double* __restrict__ ln, int64_t* scratch,
                                           int64_t scratch_stride, double* ahat_out,
                                           double* D_out, uint32_t* flags_out,
                                           uint32_t* status_out, uint32_t K) {
  __shared__ HeavyWave W;
  int64_t* gov = scratch + (int64_t)blockIdx.x * scratch_stride;
  const int64_t half = scratch_stride / 2;
  int64_t* lv = gov + half;
  uint32_t* lc = reinterpret_cast<uint32_t*>(lv + half / 2);
  const int lane = lane_id();
  for (int set = (int)blockIdx.x; set < n_sets; set += (int)gridDim.x) {
    const int64_t* x = xs[set];
    const int64_t n = ns[set];
    auto fill = [&](auto sink, uint32_t&) {
      for (int64_t i = lane; i < n; i += 64) sink(x[i]);
    };
    double a = 0.0, D = 0.0;
    uint32_t flags = 0;
    uint64_t fp;
    int64_t xmax;
    bool ok;
    heavy_core<true>(&W, n, fill, gov, lv, lc, ln, K, false, a, D, flags, fp, xmax, ok);
    if (lane == 0) {
      ahat_out[set] = a;
      D_out[set] = D;
      flags_out[set] = flags;
      status_out[set] = ok ? 0u : kErrBadValue;
    }
    wave_sync_global();
  }
}

// ---------------------------------------------------------------------------
// Table build: T[k] = F(k; alpha) = 1 - zeta(alpha, k+1)/zeta(alpha), the
// CDF of eq. (1), for k = 1..kH; then the guide table and per-cell constants.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_table(const DevCell* __restrict__ cells,
                                              double* __restrict__ tables,
                                              const double* __restrict__ ln,
                                              uint32_t* __restrict__ zero, int n_zero) {
  // the first block also clears the simulation's counters (one launch fewer)
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = (int)threadIdx.x; i < n_zero; i += (int)blockDim.x) zero[i] = 0u;
  const int cell = (int)blockIdx.y;
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x) + 1;
  if (k > kH || cells[cell].K != 0u) return;
  const double a = cells[cell].alpha;
  double suf[17];
  const int64_t xmin = cells[cell].xmin;
  if (xmin > 1) {  // T[k-1] = F(xmin + k - 1) = 1 - zeta(a, xmin + k)/zeta(a, xmin)
    const EmCoef E = em_coef(a);
    survival_head_cut(E, ln, suf);
    // zeta(a, q), q >= 2 (static indices into suf: no scratch); above a
    // cutoff of 17 every value relative to xmin^-a (survival_rel)
    auto zq = [&](int64_t q) {
      double z = 0.0;
#pragma unroll
      for (int t = 1; t <= 16; ++t)
        if (q - 1 == t) z = suf[t];
      if (xmin > 17) return survival_rel(E, q - 1, xmin);
      return q <= 17 ? z : survival_next_cut(E, q - 1, ln);
    };
    tables[(size_t)cell * kH + (k - 1)] = 1.0 - zq(xmin + k) / zq(xmin);
    return;
  }
  survival_head(a, ln, suf);
  double zk = suf[16];
#pragma unroll
  for (int t = 1; t < 16; ++t)
    if (k == t) zk = suf[t];
  if (k > 16) zk = survival_next(a, (int64_t)k, ln);
  tables[(size_t)cell * kH + (k - 1)] = 1.0 - zk / suf[0];
}

// Table of the truncated law on 1..K (Sect. 1 with a finite upper limit):
// T[k] = F(k) = 1 - Z(k)/Z(0) with Z(t) = sum_{j=t+1..K} j^-a, and T[k] = 1
// for k >= K, so a uniform never reaches the tail sampler.  The terms are
// computed in parallel; one thread forms the suffix sums from K down, in
// the order of the definition.  One workgroup per cell (pure-law cells exit).
__global__ __launch_bounds__(1024) void k_table_trunc(const DevCell* __restrict__ cells,
                                                     double* __restrict__ tables,
                                                     const double* __restrict__ ln) {
  const int cell = (int)blockIdx.x;
  const uint32_t K = cells[cell].K;
  if (K == 0u) return;
  __shared__ double w[kH + 2];  // w[j] = j^-a; then w[t + 1] = Z(t)
  const double a = cells[cell].alpha;
  const int tid = (int)threadIdx.x;
  for (int j = tid + 1; j <= (int)K; j += (int)blockDim.x) w[j] = j == 1 ? 1.0 : pow_neg(a, ln[j]);
  __syncthreads();
  if (tid == 0) {
    double z = 0.0;  // Z(K) = 0
    for (int t = (int)K - 1; t >= 0; --t) {
      const double wt = w[t + 1];
      w[t + 2] = z;  // Z(t + 1)
      z += wt;       // Z(t)
    }
    w[1] = z;
  }
  __syncthreads();
  const double z0 = w[1];
  double* T = tables + (size_t)cell * kH;
  for (int k = tid + 1; k <= kH; k += (int)blockDim.x)
    T[k - 1] = k >= (int)K ? 1.0 : 1.0 - w[k + 1] / z0;
}

// Guide entry b: the smallest k that a uniform in bin b can map to.  Bins
// b < kGA hold U in [b/(2 kGA), (b+1)/(2 kGA)); the others hold U with
// e = 1 - U in one (octave, sub-bin) cell, i.e. U in (1 - e_hi, 1 - e_lo].
// Entry kGuide is the sentinel kH.
// Guide entry b: 1 + the first index k with floor(T[k] 2^53) >= the smallest
// m of bin b (kH when none), the smallest value a uniform of the bin maps to;
// the cell's layout from its table (guide_layout).
__global__ __launch_bounds__(256) void k_guide(DevCell* __restrict__ cells,
                                              const double* __restrict__ tables,
                                              uint16_t* __restrict__ guides) {
  const int cell = (int)blockIdx.y;
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b > kGuide) return;
  const double* T = tables + (size_t)cell * kH;
  const int sh = guide_layout(T);
  int g = kH;
  if (b < kGuide) {
    const uint64_t mmin = guide_bin_min(b, sh);
    int lo = 0, hi = kH;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (table_int(T[mid]) >= mmin)
        hi = mid;
      else
        lo = mid + 1;
    }
    g = lo < kH ? lo + 1 : kH;
  }
  guides[(size_t)cell * (kGuide + 1) + b] = (uint16_t)g;
  if (b == 0) {
    DevCell& c = cells[cell];
    c.tmax = T[kH - 1];
    c.beta = c.alpha - 1.0;
    c.gm = tail_g(c.beta, (double)(c.xmin + kH));
    c.gsh = (uint32_t)sh;
  }
}

// ln k for k = 0..kH+1 (ln 0 unused, set to 0).
__global__ void k_ln_table(double* ln) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k > kH + 1) return;
  ln[k] = k == 0 ? 0.0 : log((double)k);
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Order statistics per cell: the element of rank k = floor(R num/den) in the
// ascending D values (the annex's index rule).  D >= 0, so comparing the FP64
// bit patterns as unsigned integers orders the values.  Up to kSelQ quantiles
// at a time, in three launches:
//   1. k_sel_bracket (a workgroup per cell): a sample of kSelSample values at
//      fixed positions; each quantile brackets the sample values 5 standard
//      deviations of the sample rank around its expected position.  Instead of
//      sorting the sample, a histogram of the 11 bits below the sample's common
//      high bits (with each bin's smallest and largest value) locates the bins
//      of those two ranks; the bracket [lo, hi] runs from the smallest value of
//      the lower bin to the largest of the upper (it contains the two sample
//      values, and is a single value when one value fills the bin);
//   2. k_sel_gather (many workgroups per cell, each a slice of D): counts the
//      values below each bracket and gathers the values inside it into global
//      scratch, through per-(cell, quantile) counters;
//   3. k_sel_finish (a workgroup per cell): the rank k - below is selected
//      exactly among the gathered values by radix selection (11-bit digits),
//      the quantiles side by side, each from registers when its gathered
//      values fit (kSelRegs per thread), else re-read from scratch per digit.
// If rank k falls outside its bracket, or the bracket overflows its scratch,
// the radix selection runs over all of D instead.  Both give the same element.
// ---------------------------------------------------------------------------
constexpr int kSelSample = 4096;
constexpr int kSelUnroll = 8;
constexpr int kSelRegs = 24;  // gathered values per thread of a quantile group held in registers
static_assert(kHW % 256 == 0 && kHeavyHist % 256 == 0, "build_list reads 256 bins per step");

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// The bin of a 2048-bin histogram that holds rank kk (0-based: the first bin
// whose running count exceeds kk), found by one whole wave.  `sum` is the
// lane's total of bins 32 lane .. 32 lane + 31 and `incl` the inclusive scan
// of those totals across the wave.  The lane owning the rank is found from a
// ballot; its 32 bins are then scanned across lanes 0..31 (one LDS read per
// lane instead of a walk of up to 32 dependent reads).  Returns the bin, and
// in rem the rank inside it, identical on every lane; -1 when kk is not below
// the histogram's total (then rem is kk).
__device__ __forceinline__ int rank_bin(const uint32_t* hist, uint32_t incl, uint32_t sum,
                                        int64_t kk, int lane, int64_t& rem,
                                        uint32_t* bin_count = nullptr) {
  rem = kk;
  const uint64_t hit = __ballot((int64_t)incl > kk);
  if (hit == 0ull) return -1;
  const int owner = __ffsll((long long)hit) - 1;
  const int64_t base = (int64_t)(uint32_t)__shfl((int)(incl - sum), owner, 64);
  const uint32_t h = lane < 32 ? hist[owner * 32 + lane] : 0u;
  const uint32_t s = wave_incl_scan_u32(h, lane);  // lanes 32..63 add zeros
  const uint64_t hit2 = __ballot(lane < 32 && base + (int64_t)s > kk);
  const int j = __ffsll((long long)hit2) - 1;
  rem = kk - base - (int64_t)(uint32_t)__shfl((int)(s - h), j, 64);
  if (bin_count) *bin_count = (uint32_t)__shfl((int)h, j, 64);
  return owner * 32 + j;
}

struct SelLds {
  struct {
    uint32_t hist[kSelQ][2048];  // one per quantile group; the block-wide select uses [0]
  } u;
  uint64_t prefix, mask;
  int64_t krem;
  uint64_t gprefix[kSelQ], gmask[kSelQ];
  int64_t gkrem[kSelQ];
  int gstate[kSelQ];  // per group: 0 digits to select, 1 a single value left, 2 done
};

// Exact radix selection (11-bit digits) of rank k of bits[0..R), block-wide.
// All values share the bits above `top` (the caller's bracket), which are
// given in `common`; digits of 11 bits run from bit `top` down to bit 0.
__device__ uint64_t radix_select(SelLds& L, const uint64_t* __restrict__ bits, int64_t R,
                                 int64_t k, int top, uint64_t common) {
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    const uint64_t m = top >= 63 ? 0ull : (~0ull << (top + 1));
    L.prefix = common & m;
    L.mask = m;
    L.krem = k;
  }
  __syncthreads();
  for (int hi_bit = top; hi_bit >= 0; hi_bit -= 11) {
    const int width = hi_bit + 1 < 11 ? hi_bit + 1 : 11;
    const int sh = hi_bit + 1 - width;
    const uint32_t dm = (1u << width) - 1u;
    for (int b = tid; b < 2048; b += (int)blockDim.x) L.u.hist[0][b] = 0u;
    __syncthreads();
    const uint64_t pre = L.prefix, msk = L.mask;
    const int64_t nt = (int64_t)blockDim.x;
    for (int64_t i0 = 0; i0 < R; i0 += nt * kSelUnroll) {
      uint64_t bv[kSelUnroll];
#pragma unroll
      for (int u = 0; u < kSelUnroll; ++u) {
        const int64_t i = i0 + u * nt + tid;
        bv[u] = i < R ? bits[i] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kSelUnroll; ++u) {
        const int64_t i = i0 + u * nt + tid;
        if (i < R && (bv[u] & msk) == pre) atomicAdd(&L.u.hist[0][(bv[u] >> sh) & dm], 1u);
      }
    }
    __syncthreads();
    if (wave == 0) {
      uint32_t sum = 0;
      for (int t = 0; t < 32; ++t) sum += L.u.hist[0][lane * 32 + t];
      const uint32_t incl = wave_incl_scan_u32(sum, lane);
      int64_t kk;
      const int d = rank_bin(L.u.hist[0], incl, sum, L.krem, lane, kk);
      if (lane == 0 && d >= 0) {
        L.krem = kk;
        L.prefix = pre | ((uint64_t)d << sh);
        L.mask = msk | ((uint64_t)dm << sh);
      }
    }
    __syncthreads();
  }
  return L.prefix;
}

// radix_select for up to kSelQ quantiles at once: group g (threads
// 256g..256g+255 of the 1024-thread block) selects rank k[g] of its own
// array a[g][0..n[g]), whose values share the bits above top[g] with
// common[g]; groups with act[g] false idle.  Same digits, same result as
// radix_select, with the quantiles' passes running side by side.  When the
// bin holding the rank has a single value and digits remain, the next pass
// instead finds that value (the only one matching the prefix so far) and the
// group is done.  Every barrier is reached by the whole block: the loop runs
// until no group has a pass left, finished groups idling.
__device__ void radix_select_groups(SelLds& L, const uint64_t* const (&a)[kSelQ],
                                    const int64_t (&n)[kSelQ], const int64_t (&k)[kSelQ],
                                    const int (&top)[kSelQ], const uint64_t (&common)[kSelQ],
                                    const bool (&act)[kSelQ], uint64_t (&res)[kSelQ]) {
  static_assert(kSelQ * 256 == 1024, "one 256-thread group per quantile");
  const int tid = (int)threadIdx.x, g = tid >> 8, gt = tid & 255, lane = tid & 63;
  const bool scanner = ((tid >> 6) & 3) == 0;  // the group's first wave
  // this group's parameters (static indices: the arrays stay in registers)
  const uint64_t* src = nullptr;
  int64_t cnt = 0, kg = 0;
  int topg = 0;
  uint64_t comg = 0ull;
  bool actg = false;
  int maxtop = -1;
#pragma unroll
  for (int q = 0; q < kSelQ; ++q) {
    if (q == g) {
      src = a[q];
      cnt = n[q];
      kg = k[q];
      topg = top[q];
      comg = common[q];
      actg = act[q];
    }
    if (act[q] && top[q] > maxtop) maxtop = top[q];
  }
  if (gt == 0) {
    const uint64_t m = topg >= 63 ? 0ull : (~0ull << (topg + 1));
    L.gprefix[g] = comg & m;
    L.gmask[g] = m;
    L.gkrem[g] = kg;
    L.gstate[g] = actg ? 0 : 2;
  }
  // the group's values in registers when they fit (loaded once for all digits)
  const bool inreg = actg && cnt <= (int64_t)256 * kSelRegs;
  uint64_t rv[kSelRegs];
#pragma unroll
  for (int u = 0; u < kSelRegs; ++u) {
    const int64_t i = (int64_t)u * 256 + gt;
    rv[u] = inreg && i < cnt ? src[i] : 0ull;
  }
  __syncthreads();
  uint32_t* hist = L.u.hist[g];
  for (int p = 0; maxtop - 11 * p >= 0; ++p) {
    const int hb = topg - 11 * p;
    const int st = L.gstate[g];
    const bool on = actg && hb >= 0 && st == 0;
    const bool find = actg && st == 1;
    const int width = hb + 1 < 11 ? hb + 1 : 11;
    const int sh = hb + 1 - width;
    const uint32_t dm = on ? (1u << width) - 1u : 0u;
    if (on)
      for (int b = gt; b < 2048; b += 256) hist[b] = 0u;
    __syncthreads();
    if (on && inreg) {
      const uint64_t pre = L.gprefix[g], msk = L.gmask[g];
#pragma unroll
      for (int u = 0; u < kSelRegs; ++u) {
        const int64_t i = (int64_t)u * 256 + gt;
        if (i < cnt && (rv[u] & msk) == pre) atomicAdd(&hist[(rv[u] >> sh) & dm], 1u);
      }
    } else if (on) {
      const uint64_t pre = L.gprefix[g], msk = L.gmask[g];
      for (int64_t i0 = 0; i0 < cnt; i0 += 256 * kSelUnroll) {
        uint64_t bv[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          const int64_t i = i0 + u * 256 + gt;
          bv[u] = i < cnt ? src[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          const int64_t i = i0 + u * 256 + gt;
          if (i < cnt && (bv[u] & msk) == pre) atomicAdd(&hist[(bv[u] >> sh) & dm], 1u);
        }
      }
    } else if (find) {  // exactly one value matches: it is the result
      const uint64_t pre = L.gprefix[g], msk = L.gmask[g];
      if (inreg) {
#pragma unroll
        for (int u = 0; u < kSelRegs; ++u) {
          const int64_t i = (int64_t)u * 256 + gt;
          if (i < cnt && (rv[u] & msk) == pre) L.gprefix[g] = rv[u];
        }
      } else {
        for (int64_t i = gt; i < cnt; i += 256) {
          const uint64_t v = src[i];
          if ((v & msk) == pre) L.gprefix[g] = v;
        }
      }
    }
    __syncthreads();
    if (on && scanner) {
      uint32_t sum = 0;
      for (int t = 0; t < 32; ++t) sum += hist[lane * 32 + t];
      const uint32_t incl = wave_incl_scan_u32(sum, lane);
      int64_t kk;
      uint32_t nbin = 0;
      const int d = rank_bin(hist, incl, sum, L.gkrem[g], lane, kk, &nbin);
      if (lane == 0 && d >= 0) {
        L.gkrem[g] = kk;
        L.gprefix[g] = L.gprefix[g] | ((uint64_t)d << sh);
        L.gmask[g] = L.gmask[g] | ((uint64_t)dm << sh);
        if (nbin == 1u && sh > 0) L.gstate[g] = 1;
      }
    }
    if (find && gt == 0) {
      L.gmask[g] = ~0ull;
      L.gstate[g] = 2;
    }
    __syncthreads();
    // another pass only while some group has digits or its single value left
    bool more = false;
#pragma unroll
    for (int q = 0; q < kSelQ; ++q)
      if (act[q] && (L.gstate[q] == 1 || (L.gstate[q] == 0 && top[q] - 11 * (p + 1) >= 0)))
        more = true;
    if (!more) break;
  }
#pragma unroll
  for (int q = 0; q < kSelQ; ++q) res[q] = L.gprefix[q];
  __syncthreads();
}

// Per (cell, quantile) state between the three launches.
struct SelMeta {
  uint64_t lo, hi;           // bracket (FP64 bit patterns)
  unsigned long long below;  // values below lo
  uint32_t nb;               // values gathered in [lo, hi]
  uint32_t pad;
};

__global__ __launch_bounds__(1024) void k_sel_bracket(const double* __restrict__ D,
                                                     const DevCell* __restrict__ cells, int q0,
                                                     int nq, const uint32_t* __restrict__ qnum,
                                                     const uint32_t* __restrict__ qden,
                                                     SelMeta* __restrict__ meta) {
  constexpr int kSpt = kSelSample / 1024;  // sample values per thread
  __shared__ uint32_t cnt[2048];
  __shared__ unsigned long long bmin[2048], bmax[2048];
  __shared__ uint64_t wor[16], wand[16];
  __shared__ int bin_of[2 * kSelQ];
  __shared__ int64_t rank_ab[2 * kSelQ];  // sample ranks a, b of each quantile
  __shared__ uint64_t sample[kSelSample];  // for the exact order statistics (rare case)
  __shared__ SelLds L;
  const int cell = (int)blockIdx.x;
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const DevCell c = cells[cell];
  const uint64_t* bits = reinterpret_cast<const uint64_t*>(D + c.out_off);
  const int64_t R = c.R;
  // sample ranks a = p - dl and b = p + dl of each quantile, as in the sorted
  // sample (published by the first barrier below)
  if (tid < nq) {
    const int64_t k = (int64_t)(((uint64_t)R * qnum[q0 + tid]) / qden[q0 + tid]);
    const double qf = (double)k / (double)R;
    const int64_t p = (int64_t)(qf * kSelSample);
    const int64_t dl = (int64_t)(5.0 * sqrt((double)kSelSample * qf * (1.0 - qf))) + 8;
    rank_ab[2 * tid] = p - dl;
    rank_ab[2 * tid + 1] = p + dl;
  }
  uint64_t x[kSpt];
  uint64_t o = 0ull, an = ~0ull;
#pragma unroll
  for (int t = 0; t < kSpt; ++t) {
    const uint64_t pos = (uint64_t)(tid + 1024 * t);
    x[t] = bits[(int64_t)((pos * (uint64_t)R) / kSelSample)];
    sample[pos] = x[t];
    o |= x[t];
    an &= x[t];
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    o |= shfl_xor_u64(o, m);
    an &= shfl_xor_u64(an, m);
  }
  if (lane == 0) {
    wor[wave] = o;
    wand[wave] = an;
  }
  for (int b = tid; b < 2048; b += 1024) {
    cnt[b] = 0u;
    bmin[b] = ~0ull;
    bmax[b] = 0ull;
  }
  __syncthreads();
  o = 0ull;
  an = ~0ull;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    o |= wor[w];
    an &= wand[w];
  }
  // the sample's common high bits, then an 11-bit digit below them
  const uint64_t diff = o ^ an;
  const int top = diff ? 63 - __clzll((long long)diff) : 0;
  const int sh = top > 10 ? top - 10 : 0;
#pragma unroll
  for (int t = 0; t < kSpt; ++t) {
    const int d = (int)((x[t] >> sh) & 2047u);
    atomicAdd(&cnt[d], 1u);
    atomicMin(&bmin[d], (unsigned long long)x[t]);
    atomicMax(&bmax[d], (unsigned long long)x[t]);
  }
  __syncthreads();
  // the bin holding sample rank r is the first whose running count exceeds r
  if (wave == 0) {
    uint32_t sum = 0;
    for (int t = 0; t < 32; ++t) sum += cnt[lane * 32 + t];
    const uint32_t incl = wave_incl_scan_u32(sum, lane);
    for (int r = 0; r < 2 * nq; ++r) {
      int64_t rk = rank_ab[r];
      rk = rk < 0 ? 0 : (rk > kSelSample - 1 ? kSelSample - 1 : rk);
      int64_t kk;
      const int d = rank_bin(cnt, incl, sum, rk, lane, kk);  // the sample holds 4096 > rk
      if (lane == 0) bin_of[r] = d;
    }
  }
  __syncthreads();
  // The bracket holds [sample[a], sample[b]]: the smallest value of a's bin
  // and the largest of b's.  When both ranks fall in one bin that holds more
  // than one value, sample[a] and sample[b] themselves are selected (radix
  // selection over the sample), so that a value filling ranks a..b (an atom
  // of D) still gives lo = hi.
  for (int q = 0; q < nq; ++q) {
    const int64_t a = rank_ab[2 * q], b = rank_ab[2 * q + 1];
    const int ba = bin_of[2 * q], bb = bin_of[2 * q + 1];
    uint64_t lo = a <= 0 ? 0ull : (uint64_t)bmin[ba];
    uint64_t hi = b >= kSelSample - 1 ? ~0ull : (uint64_t)bmax[bb];
    if (a > 0 && b < kSelSample - 1 && ba == bb && bmin[ba] != bmax[ba]) {
      lo = radix_select(L, sample, kSelSample, a, 63, 0ull);
      hi = radix_select(L, sample, kSelSample, b, 63, 0ull);
    }
    if (tid == 0) {
      SelMeta m;
      m.lo = lo;
      m.hi = hi;
      m.below = 0ull;
      m.nb = 0u;
      m.pad = 0u;
      meta[(size_t)cell * kSelQ + q] = m;
    }
  }
}

// Slice `slice` of cell `cell` (blocks laid out cell-major, `slices` per
// cell): values below each bracket are counted, values inside are appended
// to the quantile's gather area.  Per step of 256 x kSelUnroll values the
// workgroup takes its slots with one atomic per quantile (a wave scan of the
// threads' counts, then the four waves' totals), not one per wave and value.
__global__ __launch_bounds__(256) void k_sel_gather(const double* __restrict__ D,
                                                   const DevCell* __restrict__ cells, int nq,
                                                   int slices, int64_t chunk,
                                                   SelMeta* __restrict__ meta,
                                                   uint64_t* __restrict__ gather, int64_t gcap) {
  __shared__ uint32_t wtot[4][kSelQ];   // per wave, in-bracket values of the step
  __shared__ uint32_t wbase[4][kSelQ];  // first slot of each wave's values
  const int cell = (int)(blockIdx.x / (unsigned)slices);
  const int slice = (int)(blockIdx.x % (unsigned)slices);
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const DevCell c = cells[cell];
  const int64_t R = c.R;
  const int64_t ib = (int64_t)slice * chunk;
  if (ib >= R) return;  // the whole block
  const int64_t ie = ib + chunk < R ? ib + chunk : R;
  const uint64_t* bits = reinterpret_cast<const uint64_t*>(D + c.out_off);
  SelMeta* M = meta + (size_t)cell * kSelQ;
  uint64_t* G = gather + (size_t)cell * kSelQ * gcap;
  uint64_t lo[kSelQ], hi[kSelQ];
  uint32_t below[kSelQ];
#pragma unroll
  for (int qq = 0; qq < kSelQ; ++qq) {
    lo[qq] = qq < nq ? M[qq].lo : 0ull;
    hi[qq] = qq < nq ? M[qq].hi : 0ull;
    below[qq] = 0u;
  }
  for (int64_t i0 = ib; i0 < ie; i0 += 256 * kSelUnroll) {
    uint64_t bv[kSelUnroll];
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      const int64_t i = i0 + u * 256 + tid;
      bv[u] = i < ie ? bits[i] : 0ull;
    }
    uint32_t inm[kSelQ], incl[kSelQ], cnt[kSelQ];
#pragma unroll
    for (int qq = 0; qq < kSelQ; ++qq) {
      inm[qq] = 0u;
      cnt[qq] = 0u;
#pragma unroll
      for (int u = 0; u < kSelUnroll; ++u) {
        const bool valid = i0 + u * 256 + tid < ie;
        const uint64_t b = bv[u];
        const bool bl = qq < nq && valid && b < lo[qq];
        const bool in = qq < nq && valid && !bl && b <= hi[qq];
        below[qq] += bl ? 1u : 0u;
        inm[qq] |= in ? (1u << u) : 0u;
        cnt[qq] += in ? 1u : 0u;
      }
      incl[qq] = wave_incl_scan_u32(cnt[qq], lane);
      if (lane == 63) wtot[wave][qq] = incl[qq];
    }
    __syncthreads();
    if (tid < kSelQ) {
      uint32_t t = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        wbase[w][tid] = t;
        t += wtot[w][tid];
      }
      const uint32_t b = (tid < nq && t) ? atomicAdd(&M[tid].nb, t) : 0u;
#pragma unroll
      for (int w = 0; w < 4; ++w) wbase[w][tid] += b;
    }
    __syncthreads();
#pragma unroll
    for (int qq = 0; qq < kSelQ; ++qq) {
      if (inm[qq]) {
        uint32_t slot = wbase[wave][qq] + incl[qq] - cnt[qq];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          if (inm[qq] & (1u << u)) {
            if ((int64_t)slot < gcap) G[qq * gcap + slot] = bv[u];
            ++slot;
          }
        }
      }
    }
    __syncthreads();  // wtot and wbase are reused by the next step
  }
  // values below each bracket: one atomic per workgroup and quantile (a cell's
  // counters share a cache line, which every workgroup of the cell updates)
#pragma unroll
  for (int qq = 0; qq < kSelQ; ++qq) {
    const uint32_t w = wave_sum_u32(below[qq]);
    if (lane == 0) wtot[wave][qq] = w;
  }
  __syncthreads();
  if (tid < nq) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) t += wtot[w][tid];
    if (t) atomicAdd(&M[tid].below, (unsigned long long)t);
  }
}

__global__ __launch_bounds__(1024) void k_sel_finish(const double* __restrict__ D,
                                                    const DevCell* __restrict__ cells, int q0,
                                                    int nq, int n_q,
                                                    const uint32_t* __restrict__ qnum,
                                                    const uint32_t* __restrict__ qden,
                                                    const SelMeta* __restrict__ meta,
                                                    double* __restrict__ qout,
                                                    uint64_t* __restrict__ gather, int64_t gcap) {
  __shared__ SelLds L;
  const int cell = (int)blockIdx.x;
  const int tid = (int)threadIdx.x;
  const DevCell c = cells[cell];
  const uint64_t* bits = reinterpret_cast<const uint64_t*>(D + c.out_off);
  const uint64_t* G = gather + (size_t)cell * kSelQ * gcap;
  const SelMeta* M = meta + (size_t)cell * kSelQ;
  const int64_t R = c.R;
  const uint64_t* arr[kSelQ];
  int64_t cnt[kSelQ], rk[kSelQ];
  int tops[kSelQ];
  uint64_t com[kSelQ], res[kSelQ];
  bool grp[kSelQ], full[kSelQ];
#pragma unroll
  for (int qq = 0; qq < kSelQ; ++qq) {
    arr[qq] = G + qq * gcap;
    cnt[qq] = 0;
    rk[qq] = 0;
    tops[qq] = 0;
    com[qq] = 0ull;
    res[qq] = 0ull;
    grp[qq] = false;
    full[qq] = false;
    if (qq < nq) {
      const int64_t k = (int64_t)(((uint64_t)R * qnum[q0 + qq]) / qden[q0 + qq]);
      const SelMeta m = M[qq];
      const int64_t lo_rank = (int64_t)m.below;
      const int64_t nin = (int64_t)m.nb;
      rk[qq] = k;
      if (k >= lo_rank && k < lo_rank + nin && m.lo == m.hi) {
        res[qq] = m.lo;  // every value in the bracket equals lo (an atom of D)
      } else if (k >= lo_rank && k < lo_rank + nin && nin <= gcap) {
        const uint64_t x = m.lo ^ m.hi;
        tops[qq] = x ? 63 - __clzll((long long)x) : 0;
        com[qq] = m.lo;
        cnt[qq] = nin;
        rk[qq] = k - lo_rank;
        grp[qq] = true;
      } else {
        full[qq] = true;
      }
    }
  }
  uint64_t gres[kSelQ];
  radix_select_groups(L, arr, cnt, rk, tops, com, grp, gres);
#pragma unroll
  for (int qq = 0; qq < kSelQ; ++qq) {
    if (grp[qq]) res[qq] = gres[qq];
    if (full[qq]) res[qq] = radix_select(L, bits, R, rk[qq], 63, 0ull);
  }
  if (tid == 0) {
#pragma unroll
    for (int qq = 0; qq < kSelQ; ++qq)
      if (qq < nq) qout[cell * n_q + q0 + qq] = __longlong_as_double((long long)res[qq]);
  }
}

// count of D_b >= D_obs over the bootstrap replicates.
__global__ __launch_bounds__(256) void k_count_ge(const double* __restrict__ Db, int64_t B,
                                                 const double* __restrict__ Dobs,
                                                 unsigned long long* __restrict__ count) {
  const double d = *Dobs;
  uint32_t local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B;
       i += (int64_t)gridDim.x * blockDim.x)
    local += (Db[i] >= d) ? 1u : 0u;
  local = wave_sum_u32(local);
  if ((threadIdx.x & 63u) == 0u && local) atomicAdd(count, (unsigned long long)local);
}

// Per cell c: count of D[out_off + b] >= dobs[c], b < R (batched bootstrap).
__global__ __launch_bounds__(256) void k_count_cells(const double* __restrict__ D,
                                                    const DevCell* __restrict__ cells,
                                                    const double* __restrict__ dobs,
                                                    unsigned long long* __restrict__ counts) {
  const int cell = (int)blockIdx.y;
  const DevCell c = cells[cell];
  const double d = dobs[cell];
  uint32_t local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.R;
       i += (int64_t)gridDim.x * blockDim.x)
    local += (D[c.out_off + i] >= d) ? 1u : 0u;
  local = wave_sum_u32(local);
  if ((threadIdx.x & 63u) == 0u && local) atomicAdd(&counts[cell], (unsigned long long)local);
}

// Raw draws of replicates rep_lo.. in draw order (parity checks of the
// sampler), through the same fast path and resolution as the simulation.
__global__ __launch_bounds__(256) void k_draws(const DevCell* __restrict__ cells,
                                              const double* __restrict__ tables,
                                              const uint16_t* __restrict__ guides,
                                              int64_t rep_lo, int64_t count,
                                              int64_t* __restrict__ x,
                                              uint32_t* __restrict__ flags) {
  __shared__ uint64_t T[kH];
  __shared__ uint32_t guide[kGuide];
  const DevCell c = cells[0];
  load_cell_tables(T, guide, tables, guides, c, (int)threadIdx.x, 256);
  __syncthreads();
  const int64_t total = count * c.n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rr = t / c.n;
    const uint32_t i = (uint32_t)(t - rr * c.n);
    const uint32_t rep = (uint32_t)(rep_lo + rr);
    const Words4 w = philox4x32_10(i >> 1, rep, c.stream, 0u, c.k0, c.k1);
    const uint64_t m = (i & 1u) ? m53(w.w2, w.w3) : m53(w.w0, w.w1);
    const uint64_t timax = table_int(c.tmax);
    uint32_t fl = 0;
    int64_t v = fast_draw(m, T, guide, (int)c.gsh);
    if (v < kDeferred)
      v += c.xmin - 1;
    else
      v = resolve_entry_cut(defer_entry(m, timax, i, 0), rep, c, T, guide, fl);
    x[t] = v;
    if (fl) atomicOr(&flags[rr], fl);
  }
}

}  // namespace zpl

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime in zpl_api.cpp).
// ---------------------------------------------------------------------------
namespace zpl {

hipError_t launch_ln_table(double* ln, hipStream_t s) {
  k_ln_table<<<(kH + 2 + 255) / 256, 256, 0, s>>>(ln);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_u32<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_tables(DevCell* cells, int n_cells, double* tables, uint16_t* guides,
                         const double* ln, hipStream_t s, bool any_trunc, uint32_t* zero,
                         int n_zero) {
  if (n_cells <= 0) return hipSuccess;
  k_table<<<dim3(kH / 256, n_cells), 256, 0, s>>>(cells, tables, ln, zero, n_zero);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (any_trunc) {
    k_table_trunc<<<n_cells, 1024, 0, s>>>(cells, tables, ln);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  k_guide<<<dim3((kGuide + 1 + 255) / 256, n_cells), 256, 0, s>>>(cells, tables, guides);
  return hipGetLastError();
}

static_assert(sizeof(WaveSlot) == kWaveSlotBytes, "WaveSlot layout");

hipError_t launch_simulate(int grid, const DevCell* cells, const double* tables,
                           const uint16_t* guides, const double* ln, const Unit* units,
                           int n_units, uint32_t* queue, Outputs out, uint64_t* esc_list,
                           uint32_t* esc_count, uint32_t esc_cap, int64_t* list_v,
                           uint32_t* list_c, void* wslots, uint32_t* err, hipStream_t s) {
  if (n_units <= 0 || grid <= 0) return hipSuccess;
  k_simulate<<<grid, kBlock, 0, s>>>(cells, tables, guides, ln, units, n_units, queue, out,
                                     esc_list, esc_count, esc_cap, list_v, list_c,
                                     (WaveSlot*)wslots, err);
  return hipGetLastError();
}

hipError_t launch_heavy(int grid, const DevCell* cells, const double* tables,
                        const uint16_t* guides, const double* ln, const Unit* units,
                        int n_units, const uint64_t* esc_list, const uint32_t* esc_count,
                        uint32_t esc_cap, uint32_t* queues, Outputs out, int64_t* scratch,
                        int64_t stride, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  k_heavy<<<grid, 64 * kHeavyWaves, 0, s>>>(cells, tables, guides, ln, units, n_units, esc_list, esc_count,
                              esc_cap, queues, out, scratch, stride);
  return hipGetLastError();
}

hipError_t launch_fit(int grid, const int64_t* const* xs, const int64_t* ns, int n_sets,
                      const double* ln, int64_t* scratch, int64_t stride, double* ahat,
                      double* D, uint32_t* flags, uint32_t* status, uint32_t K, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  k_fit<<<grid, 64, 0, s>>>(xs, ns, n_sets, ln, scratch, stride, ahat, D, flags, status, K);
  return hipGetLastError();
}

hipError_t launch_fit_block(const int64_t* x, int64_t n, const double* ln, int64_t* scratch,
                            int64_t stride, double* ahat, double* D, uint32_t* flags,
                            uint32_t* status, uint32_t K, hipStream_t s) {
  k_fit_block<<<1, 64 * kFitWaves, 0, s>>>(x, n, ln, scratch, stride, ahat, D, flags, status, K);
  return hipGetLastError();
}

// Scratch of the allocation-free fit (overflow values and compact list of
// one dataset, the heavy layout), one copy per GPU for the life of the
// process.  Host code never passes this name to a kernel: it stands for the
// host-side shadow; the device address comes from noalloc_scratch_address.
static __device__ __align__(256) int64_t zpl_noalloc_scratch[kNoAllocStride];

hipError_t noalloc_scratch_address(int64_t** p) {
  return hipGetSymbolAddress((void**)p, HIP_SYMBOL(zpl_noalloc_scratch));
}

hipError_t launch_fit_scan(int grid, const int64_t* x, int64_t n, const int64_t* xmins,
                           int n_cand, const double* ln, int64_t* scratch, int64_t stride,
                           double* ahat, double* D, int64_t* ntail, uint32_t* flags,
                           uint32_t* status, hipStream_t s) {
  if (n_cand <= 0 || grid <= 0) return hipSuccess;
  k_fit_scan<<<grid, 64, 0, s>>>(x, n, xmins, n_cand, ln, scratch, stride, ahat, D, ntail,
                                 flags, status);
  return hipGetLastError();
}

hipError_t launch_select(const double* D, const DevCell* cells, int n_cells, int n_q,
                         const uint32_t* qnum, const uint32_t* qden, double* qout,
                         uint64_t* gather, int64_t gcap, int64_t maxR, int n_cu, hipStream_t s) {
  if (n_cells <= 0 || n_q <= 0) return hipSuccess;
  // the per-(cell, quantile) state follows the gather areas
  SelMeta* meta = reinterpret_cast<SelMeta*>(gather + (size_t)n_cells * kSelQ * gcap);
  // slices of at least 2,048 values, about two workgroups per compute unit
  const int64_t unit = 256 * kSelUnroll;
  int64_t slices = (2 * (int64_t)n_cu + n_cells - 1) / n_cells;
  const int64_t most = (maxR + unit - 1) / unit;
  if (slices > most) slices = most;
  if (slices < 1) slices = 1;
  int64_t chunk = (maxR + slices - 1) / slices;
  chunk = (chunk + unit - 1) / unit * unit;
  for (int q0 = 0; q0 < n_q; q0 += kSelQ) {
    const int nq = (n_q - q0) < kSelQ ? (n_q - q0) : kSelQ;
    k_sel_bracket<<<n_cells, 1024, 0, s>>>(D, cells, q0, nq, qnum, qden, meta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sel_gather<<<(unsigned)(n_cells * slices), 256, 0, s>>>(D, cells, nq, (int)slices, chunk,
                                                              meta, gather, gcap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sel_finish<<<n_cells, 1024, 0, s>>>(D, cells, q0, nq, n_q, qnum, qden, meta, qout, gather,
                                          gcap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_count_ge(const double* Db, int64_t B, const double* Dobs,
                           unsigned long long* count, hipStream_t s) {
  int grid = (int)((B + 255) / 256);
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  k_count_ge<<<grid, 256, 0, s>>>(Db, B, Dobs, count);
  return hipGetLastError();
}

hipError_t launch_count_cells(const double* D, const DevCell* cells, int n_cells,
                              const double* dobs, unsigned long long* counts, int64_t maxR,
                              hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  int gx = (int)((maxR + 255) / 256);
  if (gx > 64) gx = 64;
  if (gx < 1) gx = 1;
  k_count_cells<<<dim3(gx, n_cells), 256, 0, s>>>(D, cells, dobs, counts);
  return hipGetLastError();
}

hipError_t launch_draws(const DevCell* cell, const double* table, const uint16_t* guide,
                        int64_t rep_lo, int64_t count, int64_t* x, uint32_t* flags,
                        int64_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  int64_t g = (total + 255) / 256;
  int grid = (int)(g > 4096 ? 4096 : g);
  k_draws<<<grid, 256, 0, s>>>(cell, table, guide, rep_lo, count, x, flags);
  return hipGetLastError();
}

}  // namespace zpl
