// zpl_launch.hpp -- host launchers of the kernels in zpl_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "zpl_kernels.hpp"

namespace zpl {

hipError_t launch_ln_table(double* ln, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t s);
// CDF tables (the truncated law's only when any_trunc: a cell with K > 0)
// and packed guides; the first table block also zeroes zero[0..n_zero).
hipError_t launch_tables(DevCell* cells, int n_cells, double* tables, uint16_t* guides,
                         const double* ln, hipStream_t s, bool any_trunc = true,
                         uint32_t* zero = nullptr, int n_zero = 0);
hipError_t launch_simulate(int grid, const DevCell* cells, const double* tables,
                           const uint16_t* guides, const double* ln, const Unit* units,
                           int n_units, uint32_t* queue, Outputs out, uint64_t* esc_list,
                           uint32_t* esc_count, uint32_t esc_cap, int64_t* list_v,
                           uint32_t* list_c, void* wslots, uint32_t* err, hipStream_t s);
hipError_t launch_heavy(int grid, const DevCell* cells, const double* tables,
                        const uint16_t* guides, const double* ln, const Unit* units,
                        int n_units, const uint64_t* esc_list, const uint32_t* esc_count,
                        uint32_t esc_cap, uint32_t* queues, Outputs out, int64_t* scratch,
                        int64_t stride, hipStream_t s);
hipError_t launch_fit(int grid, const int64_t* const* xs, const int64_t* ns, int n_sets,
                      const double* ln, int64_t* scratch, int64_t stride, double* ahat,
                      double* D, uint32_t* flags, uint32_t* status, uint32_t K, hipStream_t s);
hipError_t launch_fit_block(const int64_t* x, int64_t n, const double* ln, int64_t* scratch,
                            int64_t stride, double* ahat, double* D, uint32_t* flags,
                            uint32_t* status, uint32_t K, hipStream_t s);
// Device address of the fixed scratch array of the allocation-free fit
// (kNoAllocStride int64) on the current device.
hipError_t noalloc_scratch_address(int64_t** p);
hipError_t launch_fit_scan(int grid, const int64_t* x, int64_t n, const int64_t* xmins,
                           int n_cand, const double* ln, int64_t* scratch, int64_t stride,
                           double* ahat, double* D, int64_t* ntail, uint32_t* flags,
                           uint32_t* status, hipStream_t s);
// gather: n_cells * kSelQ * gcap values, then n_cells * kSelQ * 32 bytes of
// per-(cell, quantile) state; maxR bounds every cell's R.
hipError_t launch_select(const double* D, const DevCell* cells, int n_cells, int n_q,
                         const uint32_t* qnum, const uint32_t* qden, double* qout,
                         uint64_t* gather, int64_t gcap, int64_t maxR, int n_cu, hipStream_t s);
hipError_t launch_count_ge(const double* Db, int64_t B, const double* Dobs,
                           unsigned long long* count, hipStream_t s);
hipError_t launch_count_cells(const double* D, const DevCell* cells, int n_cells,
                              const double* dobs, unsigned long long* counts, int64_t maxR,
                              hipStream_t s);
hipError_t launch_draws(const DevCell* cell, const double* table, const uint16_t* guide,
                        int64_t rep_lo, int64_t count, int64_t* x, uint32_t* flags,
                        int64_t total, hipStream_t s);

}  // namespace zpl
