// Dense comparison kernel, readout and fill launchers.
#include "bp_kernels.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

// All message slots := value (the uniform start 1/M).
__global__ __launch_bounds__(kBlock) void fill_kernel(float* dst, size_t n, float value) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = value;
}


template <int LPL, int MODE>
hipError_t go_dense(const UpdateArgs& a, hipStream_t s) {
    constexpr int CAP = kRow * LPL;
    const size_t lds = ((size_t)a.M * CAP + (kBlock / kRow) * CAP * 4) * sizeof(float);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&dense_update_kernel<LPL, MODE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int n_tiles = (a.n_slots + (kBlock / kRow) - 1) / (kBlock / kRow);
    const int grid = n_tiles < 4096 ? n_tiles : 4096;
    hipLaunchKernelGGL((dense_update_kernel<LPL, MODE>), dim3(grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int MODE>
hipError_t dense_lpl(const UpdateArgs& a, hipStream_t s) {
    switch (pick_lpl(a.M)) {
        case 1: return go_dense<1, MODE>(a, s);
        case 2: return go_dense<2, MODE>(a, s);
        case 4: return go_dense<4, MODE>(a, s);
        case 8: return go_dense<8, MODE>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int LPL>
hipError_t go_readout(const UpdateArgs& a, float* b, int* lab, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.n_slots + (kBlock / kRow) - 1) / (kBlock / kRow));
    hipLaunchKernelGGL((readout_kernel<LPL>), dim3(blocks), dim3(kBlock), 0, s, a, b, lab);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    return mode == kSum ? dense_lpl<kSum>(a, stream) : dense_lpl<kMax>(a, stream);
}

hipError_t launch_readout(const UpdateArgs& a, float* beliefs, int* labels, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    switch (pick_lpl(a.M)) {
        case 1: return go_readout<1>(a, beliefs, labels, stream);
        case 2: return go_readout<2>(a, beliefs, labels, stream);
        case 4: return go_readout<4>(a, beliefs, labels, stream);
        case 8: return go_readout<8>(a, beliefs, labels, stream);
        case 16: return go_readout<16>(a, beliefs, labels, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, dst, n, value);
    return hipGetLastError();
}

}  // namespace bpk
