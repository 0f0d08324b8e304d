// Instantiation table of the batched two-iteration kernels, included once
// per mode (bp_launch_batch_pair_sum.hip, bp_launch_batch_pair_max.hip).
#pragma once

#include "bp_batch.hpp"
#include "bp_launch.hpp"

namespace bpk {

template <int MODE, int A = 0>
hipError_t launch_batch_pair_arm(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                 hipStream_t s) {
    if constexpr (A < kBatchArms) {
        if (arm != A) return launch_batch_pair_arm<MODE, A + 1>(arm, full, L, grid, parity, s);
        if (full)
            hipLaunchKernelGGL((batch_update2_kernel<MODE, arm_g(A), arm_tw(A), true>), dim3(grid), dim3(kBlock), 0,
                               s, L, parity);
        else
            hipLaunchKernelGGL((batch_update2_kernel<MODE, arm_g(A), arm_tw(A), false>), dim3(grid), dim3(kBlock), 0,
                               s, L, parity);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace bpk
