// Host build of the library's scalar arithmetic (paper_1305_6738_amd/csrc/
// zpl_math.hpp) exposed through a C ABI, so that its logic can be checked on
// a CPU against the oracle.  Test infrastructure only.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../paper_1305_6738_amd/csrc/zpl_math.hpp"

using namespace zpl;

static std::vector<double> g_ln = [] {
  std::vector<double> v(kH + 2);
  v[0] = 0.0;
  for (int k = 1; k <= kH + 1; ++k) v[k] = std::log((double)k);
  return v;
}();

extern "C" {
void hm_philox(const uint32_t* c, const uint32_t* k, uint32_t* out) {
  Words4 w = philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1]);
  out[0] = w.w0; out[1] = w.w1; out[2] = w.w2; out[3] = w.w3;
}
int64_t hm_tail(double alpha, uint64_t seed, uint32_t stream, uint32_t rep, uint32_t i,
                uint32_t* flags) {
  const double beta = alpha - 1.0;
  return tail_draw(beta, tail_g(beta, kTailM), (uint32_t)seed, (uint32_t)(seed >> 32), i, rep,
                   stream, flags);
}
double hm_mle(double m, uint32_t* flags) { return mle_alpha(m, g_ln.data(), flags); }
double hm_mle_it(double m, uint32_t* flags, int* iters) {
  return mle_alpha(m, g_ln.data(), flags, iters);
}
double hm_mle_trunc_it(double m, uint32_t K, uint32_t* flags, int* iters) {
  return mle_alpha_trunc(m, K, g_ln.data(), flags, iters);
}
double hm_mle_hz_it(double m, int64_t xmin, uint32_t* flags, int* iters) {
  return mle_alpha_hz(m, xmin, g_ln.data(), flags, iters);
}
void hm_zeta3(double s, double* out) {
  Z3 z = zeta3(s, g_ln.data());
  out[0] = z.z0; out[1] = z.z1; out[2] = z.z2;
}
void hm_table(double alpha, double* T) {
  double suf[17];
  survival_head(alpha, g_ln.data(), suf);
  for (int k = 1; k <= kH; ++k) {
    const double zk = k <= 16 ? suf[k] : survival_next(alpha, k, g_ln.data());
    T[k - 1] = 1.0 - zk / suf[0];
  }
}
double hm_survival(double a, int64_t v) {  // zeta(a, v+1)
  double suf[17];
  survival_head(a, g_ln.data(), suf);
  return v <= 16 ? suf[v] : survival_next(a, v, g_ln.data());
}
double hm_S(const int64_t* x, int64_t n) {
  U128 S = {0, 0};
  for (int64_t i = 0; i < n; ++i) u128_add(S, ln_fixed(x[i], g_ln.data()), 0);
  return u128_to_S(S);
}
void hm_hurwitz3(double s, int64_t xmin, double* out) {
  Z3 z = hurwitz3(s, xmin, g_ln.data());
  out[0] = z.z0; out[1] = z.z1; out[2] = z.z2;
}
double hm_survival_cut(double a, int64_t v) {  // zeta(a, v+1), law with a cutoff
  const EmCoef E = em_coef(a);
  double suf[17];
  survival_head_cut(E, g_ln.data(), suf);
  return v <= 16 ? suf[v] : survival_next_cut(E, v, g_ln.data());
}
double hm_survival_rel(double a, int64_t v, int64_t xmin) {  // zeta(a, v+1) xmin^a
  return survival_rel(em_coef(a), v, xmin);
}
double hm_mle_hz(double m, int64_t xmin, uint32_t* flags) {
  return mle_alpha_hz(m, xmin, g_ln.data(), flags);
}
int64_t hm_tail_from(double alpha, int64_t xmin, uint64_t seed, uint32_t stream, uint32_t rep,
                     uint32_t i, uint32_t* flags) {
  const double beta = alpha - 1.0, m0 = (double)(xmin + kH);
  return tail_draw_from(m0, beta, tail_g(beta, m0), (uint32_t)seed, (uint32_t)(seed >> 32), i,
                        rep, stream, flags);
}
void hm_zeta3_trunc(double s, uint32_t K, double* out) {
  Z3 z = zeta3_trunc(s, K, g_ln.data());
  out[0] = z.z0; out[1] = z.z1; out[2] = z.z2;
}
void hm_zeta3_trunc_em(double s, uint32_t K, double* out) {
  Z3 z = zeta3_trunc_em(s, K, g_ln.data());
  out[0] = z.z0; out[1] = z.z1; out[2] = z.z2;
}
void hm_moments012(double z, double* out) {
  moments012(z, out[0], out[1], out[2]);
}
int hm_guide_index(uint64_t m, int sh) { return guide_index(m, sh); }
int hm_guide_refinement(uint64_t timax) { return guide_refinement(timax); }
void hm_guide_pack_all(const uint16_t* g, int sh, uint64_t timax, uint32_t* out) {
  for (int b = 0; b < kGuide; ++b) out[b] = guide_pack(g, b, sh, timax);
}
void hm_guide_index_many(const uint64_t* m, int64_t n, int sh, int32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = guide_index(m[i], sh);
}
// The guide as the simulation builds it from a table T[0..kH): g[0..kGuide]
// and the refinement; the same functions the guide kernel calls.
int hm_guide_build(const double* T, uint16_t* g) {
  const int sh = guide_layout(T);
  for (int b = 0; b <= kGuide; ++b) {
    int v = kH;
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
      v = lo < kH ? lo + 1 : kH;
    }
    g[b] = (uint16_t)v;
  }
  return sh;
}
double hm_mle_trunc(double m, uint32_t K, uint32_t* flags) {
  return mle_alpha_trunc(m, K, g_ln.data(), flags);
}
void hm_dd_exp_log(double v, double* out) {
  DD l = dd_log(v);
  DD e = dd_exp(DD{v, 0.0});
  out[0] = l.hi; out[1] = l.lo; out[2] = e.hi; out[3] = e.lo;
}
void hm_dd_exp(double hi, double lo, double* out) {
  DD e = dd_exp(DD{hi, lo});
  out[0] = e.hi; out[1] = e.lo;
}
}
