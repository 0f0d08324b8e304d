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


template <int G, int MODE>
hipError_t go_dense(const UpdateArgs& a, hipStream_t s) {
    const size_t lds = dense_lds_bytes(G, a.M, MODE);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_update_kernel<G, MODE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    constexpr int BLK = dense_block(G);
    const int n_tiles = (a.n_slots + (BLK / G) - 1) / (BLK / G);
    const int grid = n_tiles < 4096 ? n_tiles : 4096;
    hipLaunchKernelGGL((dense_update_kernel<G, MODE>), dim3(grid), dim3(BLK), lds, s, a);
    return hipGetLastError();
}

template <int MODE>
hipError_t dense_g(const UpdateArgs& a, hipStream_t s) {
    switch (lanes_for(a.M)) {
        case 4: return go_dense<4, MODE>(a, s);
        case 8: return go_dense<8, MODE>(a, s);
        case 16: return go_dense<16, MODE>(a, s);
        case 32: return go_dense<32, MODE>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G>
hipError_t go_readout(const UpdateArgs& a, float* b, int* lab, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.n_slots + (kBlock / G) - 1) / (kBlock / G));
    hipLaunchKernelGGL((readout_kernel<G>), dim3(blocks), dim3(kBlock), 0, s, a, b, lab);
    return hipGetLastError();
}

}  // namespace

size_t dense_lds_need(int M, int mode) { return dense_lds_bytes(lanes_for(M), M, mode); }

hipError_t launch_dense(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    return mode == kSum ? dense_g<kSum>(a, stream) : dense_g<kMax>(a, stream);
}

hipError_t launch_readout(const UpdateArgs& a, float* beliefs, int* labels, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    switch (lanes_for(a.M)) {
        case 4: return go_readout<4>(a, beliefs, labels, stream);
        case 8: return go_readout<8>(a, beliefs, labels, stream);
        case 16: return go_readout<16>(a, beliefs, labels, stream);
        case 32: return go_readout<32>(a, beliefs, labels, stream);
        case 64: return go_readout<64>(a, beliefs, labels, stream);
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
