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
// Inverse-CDF body search: x = min{k in 1..kH : T[k] >= U} (the ">=" rule of
// the paper's sampler).  The guide table brackets the answer; a binary search
// finishes it.  Entries k <= TL come from LDS, the rest from global memory.
// ---------------------------------------------------------------------------
template <int TL>
__device__ __forceinline__ int body_search(double U, const double* __restrict__ Ts,
                                           const double* __restrict__ Tg,
                                           const uint16_t* __restrict__ guide) {
  const int j = (int)(U * (double)kG);
  int lo = guide[j];
  int hi = (j + 1 < kG) ? (int)guide[j + 1] : kH;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double t = (mid <= TL) ? Ts[mid - 1] : Tg[mid - 1];
    if (t >= U)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

__device__ __noinline__ int64_t tail_draw_dev(double beta, double gm, uint32_t k0,
                                              uint32_t k1, uint32_t i, uint32_t rep,
                                              uint32_t stream, uint32_t* flags) {
  return tail_draw(beta, gm, k0, k1, i, rep, stream, flags);
}

template <int TL>
__device__ __forceinline__ int64_t draw_one(double U, uint32_t i, uint32_t rep,
                                            const DevCell& c, const double* __restrict__ Ts,
                                            const double* __restrict__ Tg,
                                            const uint16_t* __restrict__ guide,
                                            uint32_t& fl) {
  if (U <= c.tmax) return (int64_t)body_search<TL>(U, Ts, Tg, guide);
  return tail_draw_dev(c.beta, c.gm, c.k0, c.k1, i, rep, c.stream, &fl);
}

// ---------------------------------------------------------------------------
// KS distance (eq. 3) over the distinct values of one replicate, in
// ascending order.  With C the count of draws <= t and Z(t) = zeta(a, t+1)
// (so F(t) = 1 - Z(t)/zeta(a)), each distinct value v contributes
// |Z(v)/zeta - (n - C(v))/n| and |Z(v-1)/zeta - (n - C(v-1))/n|: between
// sample values S_n is flat and F rises, so the sup over all t is reached at
// a sample value or one below it.  Values <= 16 use the precomputed head
// suf[], larger ones the Euler-Maclaurin tail.  Src yields the distinct
// values: small(v) returns the count of v for v = 1..16 in order, then
// next_large() returns the remaining (value, count) pairs ascending.
// ---------------------------------------------------------------------------
template <class Src>
__device__ __forceinline__ double ks_distance(Src& src, double a, const double (&suf)[17],
                                              int64_t n, const double* __restrict__ ln) {
  const double z = suf[0], dn = (double)n;
  int64_t C = 0;
  double D = 0.0;
#pragma unroll
  for (int v = 1; v <= 16; ++v) {
    const uint32_t c = src.small(v);
    if (c) {
      const double t2 = fabs(suf[v - 1] / z - (double)(n - C) / dn);
      C += c;
      const double t1 = fabs(suf[v] / z - (double)(n - C) / dn);
      D = fmax(D, fmax(t1, t2));
    }
  }
  double zprev = suf[16];
  int64_t vprev = 16;
  int64_t v;
  uint32_t c;
  while (src.next_large(v, c)) {
    const double zv1 = (v - 1 == vprev) ? zprev : survival_at(a, v, ln);
    const double t2 = fabs(zv1 / z - (double)(n - C) / dn);
    C += c;
    const double zv = survival_next(a, v, ln);
    const double t1 = fabs(zv / z - (double)(n - C) / dn);
    D = fmax(D, fmax(t1, t2));
    zprev = zv;
    vprev = v;
  }
  return D;
}

// S (with the paper's all-ones rule), alpha_hat (eq. 2) and D (eq. 3).
template <class Src>
__device__ __forceinline__ void finish_replicate(Src& src, const U128& S, int64_t n,
                                                 uint32_t fl, const double* __restrict__ ln,
                                                 double& ahat, double& D, uint32_t& flags) {
  double Sd;
  if (S.lo == 0 && S.hi == 0) {  // every draw was 1: S := ln 2
    Sd = ln[2];
    fl |= kFlagAllOnes;
  } else {
    Sd = u128_to_S(S);
  }
  const double a = mle_alpha(Sd / (double)n, ln, &fl);
  double suf[17];
  survival_head(a, ln, suf);
  D = ks_distance(src, a, suf, n, ln);
  ahat = a;
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

// A compact ascending (value, count) list.
struct ListSrc {
  const int64_t* vals;
  const uint32_t* cnts;
  int len;
  int p;
  __device__ __forceinline__ uint32_t small(int v) {
    if (p < len && vals[p] == (int64_t)v) return cnts[p++];
    return 0u;
  }
  __device__ __forceinline__ bool next_large(int64_t& v, uint32_t& c) {
    if (p >= len) return false;
    v = vals[p];
    c = cnts[p];
    ++p;
    return true;
  }
};

// ---------------------------------------------------------------------------
// Wave-cooperative helpers for the wave and heavy forms.
// ---------------------------------------------------------------------------
// In-place ascending bitonic sort of a[0..P) (P a power of two) by one wave.
// Between stages: wave_sync for LDS, Barrier() for global memory.
template <class Sync>
__device__ void wave_bitonic(int64_t* a, int P, int lane, Sync sync) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < P; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int64_t x = a[i], y = a[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      sync();
    }
  }
}

// First index in the ascending a[0..n) holding a value >= v.
__device__ __forceinline__ int lower_bound_i64(const int64_t* a, int n, int64_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Builds the compact (value, count) list of one replicate from a histogram
// of values 1..nbins (hist[v-1]) and a sorted overflow array ov[0..oc),
// appending at lv/lc (length returned).  Also returns, identical on every
// lane, the exact 128-bit sum of ln x, the multiset fingerprint and the max.
struct Summary {
  U128 S;
  uint64_t fp;
  int64_t xmax;
  int len;
};

template <class Sync>
__device__ Summary build_list(const uint32_t* hist, int nbins, const int64_t* ov, int oc,
                              int64_t* lv, uint32_t* lc, int lane,
                              const double* __restrict__ ln, Sync sync) {
  U128 S = {0, 0};
  uint64_t fp = 0;
  int64_t xmax = 0;
  int len = 0;
  for (int b0 = 0; b0 < nbins; b0 += 64) {
    const int v = b0 + lane + 1;
    const uint32_t c = (v <= nbins) ? hist[v - 1] : 0u;
    if (c) {
      u128_add_mul(S, c, ln_fixed(v, ln));
      fp += (uint64_t)c * mix64((uint64_t)v);
      xmax = v;
    }
    const uint64_t m = __ballot(c != 0u);
    if (c) {
      const int pos = len + __popcll(m & lanes_below(lane));
      lv[pos] = v;
      lc[pos] = c;
    }
    len += __popcll(m);
  }
  for (int p0 = 0; p0 < oc; p0 += 64) {
    const int p = p0 + lane;
    const bool valid = p < oc;
    const int64_t v = valid ? ov[p] : 0;
    bool end = false;
    if (valid) {
      u128_add(S, ln_fixed(v, ln), 0);
      fp += mix64((uint64_t)v);
      xmax = v;
      end = (p == oc - 1) || (ov[p + 1] != v);
    }
    const uint64_t m = __ballot(end);
    if (end) {
      const int pos = len + __popcll(m & lanes_below(lane));
      lv[pos] = v;
      lc[pos] = (uint32_t)(p + 1 - lower_bound_i64(ov, oc, v));
    }
    len += __popcll(m);
  }
  sync();
  Summary s;
  s.S = wave_sum_u128(S);
  s.fp = wave_sum_u64(fp);
  s.xmax = wave_max_i64(xmax);
  s.len = len;
  return s;
}

__device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// ---------------------------------------------------------------------------
// Lane mode: one replicate per lane.
// ---------------------------------------------------------------------------
__device__ void lane_replicate(const DevCell& c, int32_t cell_id, int64_t rep, bool active,
                               uint32_t* __restrict__ hist, int64_t* __restrict__ ov,
                               int lane, const double* __restrict__ Ts,
                               const double* __restrict__ Tg,
                               const uint16_t* __restrict__ guide,
                               const double* __restrict__ ln, const Outputs& out,
                               uint64_t* esc_list, uint32_t* esc_count, uint32_t esc_cap,
                               uint32_t* err) {
  if (!active) return;
  uint32_t* h = hist + lane;
  int64_t* o = ov + lane;
#pragma unroll
  for (int b = 0; b < kHLB / 2; ++b) h[b * 64] = 0u;
  int oc = 0;
  bool esc = false;
  uint32_t fl = 0;
  const int64_t n = c.n;
  const uint32_t r = (uint32_t)rep;
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  for (uint32_t j = 0; j < nblk; ++j) {
    const Words4 w = philox4x32_10(j, r, c.stream, 0u, c.k0, c.k1);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const uint32_t i = 2u * j + (uint32_t)half;
      if (half == 1 && (int64_t)i >= n) break;
      const double U = half ? u53(w.w2, w.w3) : u53(w.w0, w.w1);
      const int64_t x = draw_one<kTL>(U, i, r, c, Ts, Tg, guide, fl);
      if (x <= kHLB) {
        const int v = (int)x - 1;
        atomicAdd(&h[(v >> 1) * 64], 1u << ((v & 1) * 16));
      } else if (oc < kCL) {
        o[oc * 64] = x;
        ++oc;
      } else {
        esc = true;
      }
    }
  }
  if (esc) {
    const uint32_t slot = atomicAdd(esc_count, 1u);
    if (slot < esc_cap)
      esc_list[slot] = ((uint64_t)(uint32_t)cell_id << 32) | r;
    else
      atomicOr(err, kErrEscOverflow);
    return;
  }
  // insertion sort of the (at most kCL) overflow values
  for (int p = 1; p < oc; ++p) {
    const int64_t v = o[p * 64];
    int q = p - 1;
    while (q >= 0 && o[q * 64] > v) {
      o[(q + 1) * 64] = o[q * 64];
      --q;
    }
    o[(q + 1) * 64] = v;
  }
  U128 S = {0, 0};
  uint64_t fp = 0;
  int64_t xmax = 0;
  for (int b = 0; b < kHLB / 2; ++b) {
    const uint32_t w = h[b * 64];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const uint32_t k = half ? (w >> 16) : (w & 0xffffu);
      const int64_t v = 2 * b + half + 1;
      if (k) {
        u128_add_mul(S, k, ln_fixed(v, ln));
        fp += (uint64_t)k * mix64((uint64_t)v);
        xmax = v;
      }
    }
  }
  for (int p = 0; p < oc; ++p) {
    const int64_t v = o[p * 64];
    u128_add(S, ln_fixed(v, ln), 0);
    fp += mix64((uint64_t)v);
    xmax = v;
  }
  LaneSrc src{h, o, oc, 17, 0};
  double a, D;
  uint32_t flags;
  finish_replicate(src, S, n, fl, ln, a, D, flags);
  write_outputs(out, c.out_off + rep, D, a, flags, fp, xmax);
}

// ---------------------------------------------------------------------------
// Wave mode: one wave draws one replicate at a time into an LDS histogram;
// finishes are deferred and run one replicate per lane.
// ---------------------------------------------------------------------------
struct WaveSlot {
  U128 S;
  uint64_t fp;
  int64_t xmax;
  uint32_t off, len, flags, esc;
};

struct WaveLds {
  uint32_t hist[kHW];
  int64_t ov[kCW];
  WaveSlot slot[64];
  uint32_t ovc;
};

struct WaveSync {
  __device__ void operator()() const { wave_sync(); }
};

__device__ void wave_batch(const DevCell& c, int32_t cell_id, int64_t r0, int nrep,
                           WaveLds* __restrict__ L, int64_t* __restrict__ lv,
                           uint32_t* __restrict__ lc, int lane,
                           const double* __restrict__ Ts, const double* __restrict__ Tg,
                           const uint16_t* __restrict__ guide, const double* __restrict__ ln,
                           const Outputs& out, uint64_t* esc_list, uint32_t* esc_count,
                           uint32_t esc_cap, uint32_t* err) {
  const int64_t n = c.n;
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  int done = 0;
  while (done < nrep) {
    // fill a batch of replicates while the list area has room for a worst case
    int q = 0;
    uint32_t used = 0;
    while (done + q < nrep && q < 64 && used + (uint32_t)(kHW + kCW) <= (uint32_t)kListCap) {
      const uint32_t r = (uint32_t)(r0 + done + q);
      for (int k = lane; k < kHW; k += 64) L->hist[k] = 0u;
      if (lane == 0) L->ovc = 0u;
      wave_sync();
      uint32_t c1 = 0, fl = 0;
      for (uint32_t j = (uint32_t)lane; j < nblk; j += 64u) {
        const Words4 w = philox4x32_10(j, r, c.stream, 0u, c.k0, c.k1);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const uint32_t i = 2u * j + (uint32_t)half;
          if (half == 1 && (int64_t)i >= n) break;
          const double U = half ? u53(w.w2, w.w3) : u53(w.w0, w.w1);
          const int64_t x = draw_one<kTL>(U, i, r, c, Ts, Tg, guide, fl);
          if (x == 1) {
            ++c1;
          } else if (x <= kHW) {
            atomicAdd(&L->hist[x - 1], 1u);
          } else {
            const uint32_t idx = atomicAdd(&L->ovc, 1u);
            if (idx < (uint32_t)kCW) L->ov[idx] = x;
          }
        }
      }
      c1 = wave_sum_u32(c1);
      fl = wave_or_u32(fl);
      if (lane == 0) L->hist[0] += c1;
      wave_sync();
      const uint32_t oc = L->ovc;
      if (oc > (uint32_t)kCW) {
        if (lane == 0) {
          const uint32_t slot = atomicAdd(esc_count, 1u);
          if (slot < esc_cap)
            esc_list[slot] = ((uint64_t)(uint32_t)cell_id << 32) | r;
          else
            atomicOr(err, kErrEscOverflow);
          L->slot[q].esc = 1u;
        }
        wave_sync();
        ++q;
        continue;
      }
      if (oc > 1) {
        const int P = next_pow2((int)oc);
        for (int k = (int)oc + lane; k < P; k += 64) L->ov[k] = INT64_MAX;
        wave_sync();
        wave_bitonic(L->ov, P, lane, WaveSync{});
      }
      const Summary s = build_list(L->hist, kHW, L->ov, (int)oc, lv + used, lc + used, lane,
                                   ln, WaveSync{});
      if (lane == 0) {
        WaveSlot& sl = L->slot[q];
        sl.S = s.S;
        sl.fp = s.fp;
        sl.xmax = s.xmax;
        sl.off = used;
        sl.len = (uint32_t)s.len;
        sl.flags = fl;
        sl.esc = 0u;
      }
      used += (uint32_t)s.len;
      wave_sync();
      ++q;
    }
    // deferred finishes, one replicate per lane
    if (lane < q) {
      const WaveSlot sl = L->slot[lane];
      if (!sl.esc) {
        ListSrc src{lv + sl.off, lc + sl.off, (int)sl.len, 0};
        double a, D;
        uint32_t flags;
        finish_replicate(src, sl.S, n, sl.flags, ln, a, D, flags);
        write_outputs(out, c.out_off + r0 + done + lane, D, a, flags, sl.fp, sl.xmax);
      }
    }
    wave_sync();
    done += q;
  }
}

// ---------------------------------------------------------------------------
// Persistent simulation kernel: workgroups pull units (a cell and up to 256
// replicates) from a global queue; the cell's table prefix and guide are
// staged in LDS when the cell changes.  Lane-mode units give one replicate to
// each lane; wave-mode units give 64 replicates to each wave.
// ---------------------------------------------------------------------------
union WaveRegion {
  struct {
    uint32_t hist[kHLB / 2 * 64];
    int64_t ov[kCL * 64];
  } lane;
  WaveLds wave;
};

__global__ __launch_bounds__(kBlock, 2) void k_simulate(
    const DevCell* __restrict__ cells, const double* __restrict__ tables,
    const uint16_t* __restrict__ guides, const double* __restrict__ ln,
    const Unit* __restrict__ units, int n_units, uint32_t* queue, Outputs out,
    uint64_t* esc_list, uint32_t* esc_count, uint32_t esc_cap, int64_t* list_v,
    uint32_t* list_c, uint32_t* err) {
  __shared__ double s_T[kTL];
  __shared__ uint16_t s_guide[kG];
  __shared__ WaveRegion s_wave[kWaves];
  __shared__ int s_unit;

  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t gwave = (int64_t)blockIdx.x * kWaves + wave;
  int64_t* lv = list_v + gwave * kListCap;
  uint32_t* lc = list_c + gwave * kListCap;
  int loaded = -1;

  for (;;) {
    if (tid == 0) s_unit = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int u = s_unit;
    if (u >= n_units) break;
    const Unit un = units[u];
    const DevCell c = cells[un.cell];
    const double* Tg = tables + (size_t)un.cell * kH;
    if (un.cell != loaded) {
      const uint16_t* g = guides + (size_t)un.cell * kG;
      for (int k = tid; k < kTL; k += kBlock) s_T[k] = Tg[k];
      for (int k = tid; k < kG; k += kBlock) s_guide[k] = g[k];
      loaded = un.cell;
      __syncthreads();
    }
    const int first = wave * 64;
    if (c.mode == kModeLane) {
      const int idx = first + lane;
      lane_replicate(c, un.cell, un.r0 + idx, idx < un.count, s_wave[wave].lane.hist,
                     s_wave[wave].lane.ov, lane, s_T, Tg, s_guide, ln, out, esc_list,
                     esc_count, esc_cap, err);
    } else if (first < un.count) {
      const int nrep = (un.count - first) < 64 ? (un.count - first) : 64;
      wave_batch(c, un.cell, un.r0 + first, nrep, &s_wave[wave].wave, lv, lc, lane, s_T, Tg,
                 s_guide, ln, out, esc_list, esc_count, esc_cap, err);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Heavy form: one wave per workgroup, the whole table in LDS, values above
// kHeavyHist in per-wave global scratch (sorted there).  Runs the planned
// heavy units, then every replicate that overflowed the lane or wave form.
// ---------------------------------------------------------------------------
struct BlockSync {
  __device__ void operator()() const { __syncthreads(); }
};

struct HeavyLds {
  double T[kH];
  uint16_t guide[kG];
  uint32_t hist[kHeavyHist];
  uint32_t ovc;
  int item;
};

// Draw source for the heavy form: the Philox stream of (cell, replicate).
struct DrawGen {
  const DevCell* c;
  const HeavyLds* L;
  uint32_t rep;
  __device__ __forceinline__ int64_t operator()(uint32_t i, const Words4& w, int half,
                                               uint32_t& fl) const {
    const double U = half ? u53(w.w2, w.w3) : u53(w.w0, w.w1);
    return draw_one<kH>(U, i, rep, *c, L->T, L->T, L->guide, fl);
  }
};

// Histogram/overflow fill, sort, compact list and finish of one replicate by
// one wave (blockDim == 64).  `values(i)` gives draw i.
template <class Fill>
__device__ void heavy_core(HeavyLds* L, int64_t n, Fill fill, int64_t* gov, int64_t* lv,
                           uint32_t* lc, const double* __restrict__ ln, uint32_t fl_in,
                           double& a, double& D, uint32_t& flags, uint64_t& fp,
                           int64_t& xmax, bool& ok) {
  const int lane = lane_id();
  for (int k = lane; k < kHeavyHist; k += 64) L->hist[k] = 0u;
  if (lane == 0) L->ovc = 0u;
  __syncthreads();
  uint32_t c1 = 0, fl = fl_in;
  bool bad = false;
  fill([&](int64_t x) {
    if (x < 1) {
      bad = true;
    } else if (x == 1) {
      ++c1;
    } else if (x <= kHeavyHist) {
      atomicAdd(&L->hist[x - 1], 1u);
    } else {
      const uint32_t idx = atomicAdd(&L->ovc, 1u);
      gov[idx] = x;
    }
  }, fl);
  c1 = wave_sum_u32(c1);
  fl = wave_or_u32(fl);
  const uint32_t anybad = wave_or_u32(bad ? 1u : 0u);
  if (lane == 0) L->hist[0] += c1;
  __syncthreads();
  ok = (anybad == 0u);
  if (!ok) return;
  const int oc = (int)L->ovc;
  if (oc > 1) {
    const int P = next_pow2(oc);
    for (int k = oc + lane; k < P; k += 64) gov[k] = INT64_MAX;
    __syncthreads();
    wave_bitonic(gov, P, lane, BlockSync{});
  }
  const Summary s = build_list(L->hist, kHeavyHist, gov, oc, lv, lc, lane, ln, BlockSync{});
  __syncthreads();
  ListSrc src{lv, lc, s.len, 0};
  finish_replicate(src, s.S, n, fl, ln, a, D, flags);
  fp = s.fp;
  xmax = s.xmax;
}

__device__ void heavy_load_table(HeavyLds* L, const double* T, const uint16_t* g) {
  for (int k = lane_id(); k < kH; k += 64) L->T[k] = T[k];
  for (int k = lane_id(); k < kG; k += 64) L->guide[k] = g[k];
  __syncthreads();
}

__device__ void heavy_replicate(HeavyLds* L, const DevCell& c, uint32_t rep, int64_t* gov,
                                int64_t* lv, uint32_t* lc, const double* __restrict__ ln,
                                const Outputs& out) {
  const int lane = lane_id();
  const int64_t n = c.n;
  const uint32_t nblk = (uint32_t)((n + 1) >> 1);
  DrawGen gen{&c, L, rep};
  auto fill = [&](auto sink, uint32_t& fl) {
    for (uint32_t j = (uint32_t)lane; j < nblk; j += 64u) {
      const Words4 w = philox4x32_10(j, rep, c.stream, 0u, c.k0, c.k1);
      sink(gen(2u * j, w, 0, fl));
      if ((int64_t)(2u * j + 1u) < n) sink(gen(2u * j + 1u, w, 1, fl));
    }
  };
  double a, D;
  uint32_t flags;
  uint64_t fp;
  int64_t xmax;
  bool ok;
  heavy_core(L, n, fill, gov, lv, lc, ln, 0u, a, D, flags, fp, xmax, ok);
  if (lane == 0) write_outputs(out, c.out_off + rep, D, a, flags, fp, xmax);
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_heavy(
    const DevCell* __restrict__ cells, const double* __restrict__ tables,
    const uint16_t* __restrict__ guides, const double* __restrict__ ln,
    const Unit* __restrict__ units, int n_units, const uint64_t* __restrict__ esc_list,
    const uint32_t* __restrict__ esc_count, uint32_t esc_cap, uint32_t* queues,
    Outputs out, int64_t* scratch, int64_t scratch_stride) {
  __shared__ HeavyLds L;
  int64_t* gov = scratch + (int64_t)blockIdx.x * scratch_stride;
  // list area after the overflow area: values then counts
  const int64_t half = scratch_stride / 2;
  int64_t* lv = gov + half;
  uint32_t* lc = reinterpret_cast<uint32_t*>(lv + half / 2);
  int loaded = -1;
  // planned heavy units
  for (;;) {
    if (threadIdx.x == 0) L.item = (int)atomicAdd(&queues[0], 1u);
    __syncthreads();
    const int u = L.item;
    __syncthreads();
    if (u >= n_units) break;
    const Unit un = units[u];
    const DevCell c = cells[un.cell];
    if (un.cell != loaded) {
      heavy_load_table(&L, tables + (size_t)un.cell * kH, guides + (size_t)un.cell * kG);
      loaded = un.cell;
    }
    for (int k = 0; k < un.count; ++k)
      heavy_replicate(&L, c, (uint32_t)(un.r0 + k), gov, lv, lc, ln, out);
  }
  // replicates that overflowed the lane or wave form
  const uint32_t ne = *esc_count < esc_cap ? *esc_count : esc_cap;
  for (;;) {
    if (threadIdx.x == 0) L.item = (int)atomicAdd(&queues[1], 1u);
    __syncthreads();
    const uint32_t e = (uint32_t)L.item;
    __syncthreads();
    if (e >= ne) break;
    const uint64_t code = esc_list[e];
    const int cell = (int)(code >> 32);
    const uint32_t rep = (uint32_t)code;
    const DevCell c = cells[cell];
    if (cell != loaded) {
      heavy_load_table(&L, tables + (size_t)cell * kH, guides + (size_t)cell * kG);
      loaded = cell;
    }
    heavy_replicate(&L, c, rep, gov, lv, lc, ln, out);
  }
}

// ---------------------------------------------------------------------------
// Dataset fit: S, alpha_hat and D of caller data x[0..n) (one wave per
// dataset).  Same histogram/list/finish arithmetic as the simulated
// replicates, so identical multisets give bit-identical results.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_fit(const int64_t* const* __restrict__ xs,
                                           const int64_t* __restrict__ ns, int n_sets,
                                           const double* __restrict__ ln, int64_t* scratch,
                                           int64_t scratch_stride, double* ahat_out,
                                           double* D_out, uint32_t* flags_out,
                                           uint32_t* status_out) {
  __shared__ HeavyLds L;
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
    heavy_core(&L, n, fill, gov, lv, lc, ln, 0u, a, D, flags, fp, xmax, ok);
    if (lane == 0) {
      ahat_out[set] = a;
      D_out[set] = D;
      flags_out[set] = flags;
      status_out[set] = ok ? 0u : kErrBadValue;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Table build: T[k] = F(k; alpha) = 1 - zeta(alpha, k+1)/zeta(alpha), the
// CDF of eq. (1), for k = 1..kH; then the guide table and per-cell constants.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_table(const DevCell* __restrict__ cells,
                                              double* __restrict__ tables,
                                              const double* __restrict__ ln) {
  const int cell = (int)blockIdx.y;
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x) + 1;
  if (k > kH) return;
  const double a = cells[cell].alpha;
  double suf[17];
  survival_head(a, ln, suf);
  double zk = suf[16];
#pragma unroll
  for (int t = 1; t < 16; ++t)
    if (k == t) zk = suf[t];
  if (k > 16) zk = survival_next(a, (int64_t)k, ln);
  tables[(size_t)cell * kH + (k - 1)] = 1.0 - zk / suf[0];
}

__global__ __launch_bounds__(256) void k_guide(DevCell* __restrict__ cells,
                                              const double* __restrict__ tables,
                                              uint16_t* __restrict__ guides) {
  const int cell = (int)blockIdx.y;
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= kG) return;
  const double* T = tables + (size_t)cell * kH;
  const double target = (double)j / (double)kG;
  int lo = 0, hi = kH;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (T[mid] >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  guides[(size_t)cell * kG + j] = (uint16_t)(lo < kH ? lo + 1 : kH);
  if (j == 0) {
    DevCell& c = cells[cell];
    c.tmax = T[kH - 1];
    c.beta = c.alpha - 1.0;
    c.gm = tail_g(c.beta, kTailM);
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
// Order statistics per cell: the element of rank floor(R num/den) in the
// ascending D values (the annex's index rule), by radix selection on the
// FP64 bit patterns (D >= 0, so bit order is numeric order).  One workgroup
// per (cell, quantile).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_select(const double* __restrict__ D,
                                               const DevCell* __restrict__ cells, int n_q,
                                               const uint32_t* __restrict__ qnum,
                                               const uint32_t* __restrict__ qden,
                                               double* __restrict__ qout) {
  __shared__ uint32_t hist[2048];
  __shared__ uint32_t part[256];
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ int64_t s_k;
  const int cell = (int)blockIdx.x / n_q;
  const int qi = (int)blockIdx.x % n_q;
  const int tid = (int)threadIdx.x;
  const DevCell c = cells[cell];
  const uint64_t* bits = reinterpret_cast<const uint64_t*>(D + c.out_off);
  const int64_t R = c.R;
  if (tid == 0) {
    s_k = (int64_t)(((uint64_t)R * (uint64_t)qnum[qi]) / (uint64_t)qden[qi]);
    s_prefix = 0;
    s_mask = 0;
  }
  const int shifts[6] = {53, 42, 31, 20, 9, 0};
  const int widths[6] = {11, 11, 11, 11, 11, 9};
  for (int pass = 0; pass < 6; ++pass) {
    const int sh = shifts[pass];
    const uint32_t dm = (1u << widths[pass]) - 1u;
    for (int b = tid; b < 2048; b += 256) hist[b] = 0u;
    __syncthreads();
    const uint64_t prefix = s_prefix, mask = s_mask;
    for (int64_t i = tid; i < R; i += 256) {
      const uint64_t b = bits[i];
      if ((b & mask) == prefix) atomicAdd(&hist[(b >> sh) & dm], 1u);
    }
    __syncthreads();
    uint32_t sum = 0;
    for (int b = 0; b < 8; ++b) sum += hist[tid * 8 + b];
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
      int64_t k = s_k;
      int t = 0;
      while (t < 255 && (int64_t)part[t] <= k) {
        k -= part[t];
        ++t;
      }
      int d = t * 8;
      while (d < t * 8 + 7 && (int64_t)hist[d] <= k) {
        k -= hist[d];
        ++d;
      }
      s_k = k;
      s_prefix = prefix | ((uint64_t)d << sh);
      s_mask = mask | ((uint64_t)dm << sh);
    }
    __syncthreads();
  }
  if (tid == 0) qout[cell * n_q + qi] = __longlong_as_double((long long)s_prefix);
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

// Raw draws of replicates rep_lo.. in draw order (parity checks of the
// sampler).  Table read from global memory.
__global__ void k_draws(const DevCell* __restrict__ cells, const double* __restrict__ tables,
                        const uint16_t* __restrict__ guides, int64_t rep_lo, int64_t count,
                        int64_t* __restrict__ x, uint32_t* __restrict__ flags) {
  const DevCell c = cells[0];
  const int64_t total = count * c.n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rr = t / c.n;
    const uint32_t i = (uint32_t)(t - rr * c.n);
    const uint32_t rep = (uint32_t)(rep_lo + rr);
    const Words4 w = philox4x32_10(i >> 1, rep, c.stream, 0u, c.k0, c.k1);
    const double U = (i & 1u) ? u53(w.w2, w.w3) : u53(w.w0, w.w1);
    uint32_t fl = 0;
    x[t] = draw_one<0>(U, i, rep, c, tables, tables, guides, fl);
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
                         const double* ln, hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  k_table<<<dim3(kH / 256, n_cells), 256, 0, s>>>(cells, tables, ln);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_guide<<<dim3(kG / 256, n_cells), 256, 0, s>>>(cells, tables, guides);
  return hipGetLastError();
}

hipError_t launch_simulate(int grid, const DevCell* cells, const double* tables,
                           const uint16_t* guides, const double* ln, const Unit* units,
                           int n_units, uint32_t* queue, Outputs out, uint64_t* esc_list,
                           uint32_t* esc_count, uint32_t esc_cap, int64_t* list_v,
                           uint32_t* list_c, uint32_t* err, hipStream_t s) {
  if (n_units <= 0 || grid <= 0) return hipSuccess;
  k_simulate<<<grid, kBlock, 0, s>>>(cells, tables, guides, ln, units, n_units, queue, out,
                                     esc_list, esc_count, esc_cap, list_v, list_c, err);
  return hipGetLastError();
}

hipError_t launch_heavy(int grid, const DevCell* cells, const double* tables,
                        const uint16_t* guides, const double* ln, const Unit* units,
                        int n_units, const uint64_t* esc_list, const uint32_t* esc_count,
                        uint32_t esc_cap, uint32_t* queues, Outputs out, int64_t* scratch,
                        int64_t stride, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  k_heavy<<<grid, 64, 0, s>>>(cells, tables, guides, ln, units, n_units, esc_list, esc_count,
                              esc_cap, queues, out, scratch, stride);
  return hipGetLastError();
}

hipError_t launch_fit(int grid, const int64_t* const* xs, const int64_t* ns, int n_sets,
                      const double* ln, int64_t* scratch, int64_t stride, double* ahat,
                      double* D, uint32_t* flags, uint32_t* status, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  k_fit<<<grid, 64, 0, s>>>(xs, ns, n_sets, ln, scratch, stride, ahat, D, flags, status);
  return hipGetLastError();
}

hipError_t launch_select(const double* D, const DevCell* cells, int n_cells, int n_q,
                         const uint32_t* qnum, const uint32_t* qden, double* qout,
                         hipStream_t s) {
  if (n_cells <= 0 || n_q <= 0) return hipSuccess;
  k_select<<<n_cells * n_q, 256, 0, s>>>(D, cells, n_q, qnum, qden, qout);
  return hipGetLastError();
}

hipError_t launch_count_ge(const double* Db, int64_t B, const double* Dobs,
                           unsigned long long* count, hipStream_t s) {
  int grid = (int)((B + 255) / 256);
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  k_count_ge<<<grid, 256, 0, s>>>(Db, B, Dobs, count);
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
