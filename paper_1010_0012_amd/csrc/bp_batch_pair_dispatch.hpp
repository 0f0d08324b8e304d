// Instantiation table of the batched two-iteration kernels, included once
// per mode (bp_launch_batch_pair_sum.hip, bp_launch_batch_pair_sumf.hip,
// bp_launch_batch_pair_max.hip).
#pragma once

#include "bp_batch.hpp"
#include "bp_launch.hpp"

namespace bpk {

// full: every instance of L has M = 4G.  With L.rows and one workgroup per
// range (grid == L.blocks_end[last]), the row-block kernel runs over its own
// grid of L.rows_end[last] workgroups; otherwise the per-range kernel over
// `grid`.  Float32 arithmetic exists for full launches only, and takes the
// single-grid float32 launch's default cap of 4 workgroups per CU (LDS it
// does not use).
template <int MODE, int A = 0>
hipError_t launch_batch_pair_arm(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                 hipStream_t s) {
    if constexpr (A < kBatchArms) {
        if (arm != A) return launch_batch_pair_arm<MODE, A + 1>(arm, full, L, grid, parity, s);
        const bool one_per_range = L.passes == 1 && (int)grid == L.blocks_end[L.n_inst - 1];
        const size_t lds = MODE == kSumF32 ? lds_cap_bytes(4) : 0;
        if (full && L.rows && one_per_range) {
            hipLaunchKernelGGL((batch_update2_rows_kernel<MODE, arm_g(A), arm_tw(A)>),
                               dim3((unsigned)L.rows_end[L.n_inst - 1]), dim3(kBlock), lds, s, L, parity);
        } else if (full) {
            hipLaunchKernelGGL((batch_update2_kernel<MODE, arm_g(A), arm_tw(A), true>), dim3(grid), dim3(kBlock), lds,
                               s, L, parity);
        } else if constexpr (MODE == kSumF32) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((batch_update2_kernel<MODE, arm_g(A), arm_tw(A), false>), dim3(grid), dim3(kBlock), 0,
                               s, L, parity);
        }
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace bpk
