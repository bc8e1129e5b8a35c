// zpl_kernels.hpp -- device-side data layout shared by the kernels and the
// host runtime of libzpl (not part of the public C ABI).
#pragma once

#include <stdint.h>

namespace zpl {

// Guide table: g[j] = min{k : T[k] >= j/kG}, so the search for U starts at
// g[floor(U kG)] and ends by g[floor(U kG) + 1].
constexpr int kG = 2048;

// Simulation kernel geometry: 4 wave64 per workgroup.
constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
// Leading CDF entries kept in LDS by the lane/wave kernel (later ones are read
// from the global table, through the caches).
constexpr int kTL = 512;
// Lane mode: one replicate per lane; per-lane histogram of values 1..kHLB
// (16-bit counters packed two per dword) plus a per-lane list of up to kCL
// larger values.  A replicate with more is redone by the heavy kernel.
constexpr int kHLB = 64;
constexpr int kCL = 16;
// Wave mode: one replicate per wave at a time; histogram of values 1..kHW
// plus up to kCW larger values in LDS; finishes run one replicate per lane.
constexpr int kHW = 1024;
constexpr int kCW = 1024;
// Compact (value, count) list capacity per wave for deferred finishes.
constexpr int kListCap = 16 * (kHW + kCW);
// Heavy kernel: one wave per workgroup, whole table in LDS, larger values in
// a per-wave global scratch area.
constexpr int kHeavyHist = 1024;

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

}  // namespace zpl
