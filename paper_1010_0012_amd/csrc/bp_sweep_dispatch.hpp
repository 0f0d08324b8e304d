// Instantiation table and dispatch of the sweep-pass kernels, included once
// per mode (bp_launch_sweep_sum.hip, bp_launch_sweep_sumf.hip,
// bp_launch_sweep_max.hip).
#pragma once

#include "bp_launch.hpp"
#include "bp_sparse_dispatch.hpp"
#include "bp_sweep.hpp"

namespace bpk {

template <int G, int TW, int MODE, int KIND, bool FULL>
hipError_t go_sweep_full(const UpdateArgs& a, hipStream_t s) {
    const size_t lds = sweep_lds_bytes(G, a.M, MODE, KIND);
    const void* fn = reinterpret_cast<const void*>(&sweep_pass_kernel<G, TW, MODE, KIND, FULL>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int n_lines = (a.dir == kLeft || a.dir == kRight) ? a.H : a.W;
    constexpr int LPB = kSweepBlock / G;
    const unsigned blocks = (unsigned)((n_lines + LPB - 1) / LPB) * (a.both ? 2 : 1);
    hipLaunchKernelGGL((sweep_pass_kernel<G, TW, MODE, KIND, FULL>), dim3(blocks), dim3(kSweepBlock), lds, s, a);
    return hipGetLastError();
}

// FULL (M == 4G) is a template parameter: loads, stores and normalisation
// then carry no per-label bounds.
template <int G, int TW, int MODE, int KIND>
hipError_t go_sweep(const UpdateArgs& a, hipStream_t s) {
    if constexpr (MODE == kSumF32) {
        return a.M == G * kLpl ? go_sweep_full<G, TW, MODE, KIND, true>(a, s) : hipErrorInvalidValue;
    } else {
        return a.M == G * kLpl ? go_sweep_full<G, TW, MODE, KIND, true>(a, s)
                               : go_sweep_full<G, TW, MODE, KIND, false>(a, s);
    }
}

template <int G, int MODE, int I = 0>
hipError_t sweep_tw(const UpdateArgs& a, int tw, hipStream_t s) {
    constexpr int n = sizeof(TwList<G>::v) / sizeof(int);
    if constexpr (I < n) {
        constexpr int TW = TwList<G>::v[I];
        if (tw == TW) {
            if constexpr (MODE == kMax)
                if (a.eq10) return go_sweep<G, TW, kMax, kSweepRegEq10>(a, s);
            return go_sweep<G, TW, MODE, kSweepReg>(a, s);
        }
        return sweep_tw<G, MODE, I + 1>(a, tw, s);
    } else if constexpr (MODE == kSumF32) {
        return hipErrorInvalidValue;  // float32 arithmetic: register windows only
    } else {
        if (a.eq10) return hipErrorInvalidValue;  // Eq. 10 beyond the register windows runs the general kernel
        return go_sweep<G, 0, MODE, kSweepLds>(a, s);
    }
}

template <int G, int MODE>
hipError_t sweep_g(const UpdateArgs& a, bool dense, hipStream_t s) {
    if (dense) {
        if constexpr (G <= 32 && MODE != kSumF32) return go_sweep<G, 0, MODE, kSweepDense>(a, s);
        else return hipErrorInvalidValue;
    }
    return sweep_tw<G, MODE>(a, sparse_tw(a.M, a.T), s);
}

template <int MODE>
hipError_t dispatch_sweep(const UpdateArgs& a, bool dense, hipStream_t s) {
    switch (lanes_for(a.M)) {
        case 4: return sweep_g<4, MODE>(a, dense, s);
        case 8: return sweep_g<8, MODE>(a, dense, s);
        case 16: return sweep_g<16, MODE>(a, dense, s);
        case 32: return sweep_g<32, MODE>(a, dense, s);
        case 64: return sweep_g<64, MODE>(a, dense, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bpk
