// zpl_kernels.hpp -- device-side data layout shared by the kernels and the
// host runtime of libzpl (not part of the public C ABI).
#pragma once

#include <stdint.h>

namespace zpl {

// Two-part guide table over U.  For U < 1/2: kGA bins uniform in U.  For
// U > 1/2: bins on e = 1 - U (exact in FP64), one per (octave of e, top
// kGBits + gsh mantissa bits), ordered so that the bin index increases with
// U.  Entry g[b] is the smallest k a uniform in bin b can map to, so U in bin
// b maps into [g[b], g[b+1]].  On the Zipf law the survival is close to a
// power of k, so log-scale bins keep most brackets one or two entries wide.
// gsh (0..kGuideShMax, per cell) refines the bins when the table's part of
// U > 1/2 spans few octaves of e (heavy tails: at alpha = 1.2 the table ends
// at e = 0.17, two octaves): the 3,328 entries then cover 52 >> gsh octaves,
// and indices of deeper octaves (tail draws) are clamped to the last entry.
// gsh = kGuideUniform selects a uniform layout instead, for a table whose
// support is bounded (the truncated law: no tail) and spread out: 2048 bins
// uniform in U (bin m >> 42, entries from 2048 on unused).
constexpr int kGuideShMax = 4;
constexpr int kGuideUniform = 8;
constexpr int kGA = 256;
constexpr int kGBits = 6;
constexpr int kOctaves = 52;  // e in [2^-53, 1/2)
constexpr int kGuide = kGA + (kOctaves << kGBits);

// Simulation kernel geometry: 8 wave64 per workgroup share the CDF table and
// the guide in LDS.
constexpr int kWaves = 12;  // three per SIMD
constexpr int kBlock = 64 * kWaves;
// Lane form: one replicate per lane; per-lane histogram of values 1..kHLB
// (16-bit counters packed two per dword) plus a per-lane list of up to
// kLaneCap larger values in the wave's global scratch (a replicate with more
// is redone by the heavy form).
constexpr int kHLB = 48;
constexpr int kLaneCap = 128;
// Wave form: one replicate per wave at a time; histogram of values 1..kHW
// plus up to kCW larger values in LDS; finishes run one replicate per lane.
constexpr int kHW = 1024;
constexpr int kCW = 248;
// Compact (value, count) list capacity per wave for deferred finishes.
constexpr int kListCap = 16 * (kHW + kCW);
// Heavy form: 4 wave64 per workgroup, values above kHeavyHist in per-wave
// global scratch (sorted there).
constexpr int kHeavyWaves = 4;
constexpr int kHeavyHist = 1024;
// Allocation-free fit: the overflow values and the compact list of one
// dataset of up to kNoAllocMaxN values live in a fixed device array of
// kNoAllocStride int64 (the heavy layout's stride for that n:
// 2 * max(2^20, 2 * (kHeavyHist + 2^20))).
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 20;
constexpr int64_t kNoAllocStride = 2 * (2 * ((int64_t)kHeavyHist + kNoAllocMaxN));

// Quantiles per selection pass and the per-(cell, quantile) capacity of the
// bracket gather scratch.
constexpr int kSelQ = 4;
constexpr int64_t kSelGather = 32768;
// Size of the per-replicate record of a wave-form batch (global scratch,
// 64 per wave).
constexpr int kWaveSlotBytes = 48;

enum Mode : uint32_t { kModeLane = 0, kModeWave = 1, kModeHeavy = 2 };

struct DevCell {
  double alpha;   // exponent the draws use
  double beta;    // alpha - 1
  double gm;      // tail acceptance constant g(kH + 1)
  double tmax;    // T[kH], written by the guide kernel
  int64_t n;      // draws per replicate
  int64_t R;      // replicates
  int64_t out_off;  // offset of replicate 0 in the per-replicate outputs
  uint32_t k0, k1;  // Philox key = seed
  uint32_t stream;  // Philox counter word 2
  uint32_t mode;    // Mode
  uint32_t K;       // 0: the pure law; else the truncated law on 1..K
  uint32_t gsh;     // guide refinement: 2^(kGBits + gsh) bins per octave of 1 - U
  int64_t xmin;     // lower cutoff of the pure law (1: none); values >= xmin
};

struct Unit {
  int32_t cell;
  int32_t count;  // replicates in this unit
  int64_t r0;     // first replicate
};

struct Outputs {
  double* D;
  double* ahat;
  uint32_t* flags;
  uint64_t* fp;
  int64_t* xmax;
};

// Error bits written by kernels into the context's error word.
constexpr uint32_t kErrEscOverflow = 1u;
constexpr uint32_t kErrBadValue = 2u;
constexpr uint32_t kErrNoTail = 4u;  // no value at or above the cutoff (xmin scan)

}  // namespace zpl
