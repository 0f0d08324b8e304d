// Dense comparison kernel, readout and fill launchers.
#include <algorithm>
#include <atomic>

#include "bp_kernels.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

// All message slots := value (the uniform start 1/M).
__global__ __launch_bounds__(kBlock) void fill_kernel(float* dst, size_t n, float value) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = value;
}

// One thread per unary row; a bad row sets the flag (every writer stores 1).
__global__ __launch_bounds__(kBlock) void validate_unary_kernel(const float* g, int N, int M, int* flag) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= N) return;
    const float* row = g + (size_t)p * M;
    bool ok = true, any = false;
    for (int x = 0; x < M; ++x) {
        const float v = row[x];
        ok = ok && isfinite(v) && v >= 0.0f;
        any = any || v > 0.0f;
    }
    if (!ok || !any) *flag = 1;
}

// n4 float4 stores (dst 16-byte aligned).
__global__ __launch_bounds__(kBlock) void fill4_kernel(v4f* dst, size_t n4, float value) {
    const v4f v = {value, value, value, value};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock) dst[i] = v;
}

// One thread per (border slot, label): slots [0, H) are the left slots of
// column 0, [H, 2H) the right slots of column W-1, [2H, 2H+W) the up slots of
// row 0, [2H+W, 2H+2W) the down slots of row H-1.
__global__ __launch_bounds__(kBlock) void fill_border_kernel(float* msg, int H, int W, int M, float value) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (size_t)2 * (H + W) * M) return;
    const int s = (int)(i / M), x = (int)(i - (size_t)s * M);
    int k, p;
    if (s < H) { k = kLeft; p = s * W; }
    else if (s < 2 * H) { k = kRight; p = (s - H) * W + W - 1; }
    else if (s < 2 * H + W) { k = kUp; p = s - 2 * H; }
    else { k = kDown; p = (H - 1) * W + (s - 2 * H - W); }
    msg[((size_t)k * H * W + p) * M + x] = value;
}


template <int G, int MODE>
hipError_t go_dense(const UpdateArgs& a, hipStream_t s) {
    if constexpr (MODE == kSum && (G == 8 || G == 16)) {
        if (a.M == 4 * G) {  // Eq. 2 on the matrix cores
            constexpr size_t lds = dense_mfma_lds_bytes<G>();
            if (lds > 64 * 1024) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_mfma_kernel<G>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return e;
            }
            const int n_tiles = (a.n_slots + (kBlock / G) - 1) / (kBlock / G);
            const int grid = n_tiles < 4096 ? n_tiles : 4096;
            hipLaunchKernelGGL((dense_mfma_kernel<G>), dim3(grid), dim3(kBlock), lds, s, a);
            return hipGetLastError();
        }
    }
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

size_t lds_cap_bytes(int n) {
    constexpr int kMaxDevices = 64;
    static std::atomic<int> lds_per_cu[kMaxDevices];  // 0: not yet queried
    int dev = 0;
    if (n < 1 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    int lds = lds_per_cu[dev].load(std::memory_order_relaxed);
    if (lds == 0) {
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            lds <= 0)
            return 0;
        lds_per_cu[dev].store(lds, std::memory_order_relaxed);
    }
    int per_block = 0;
    if (hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    // n workgroups of floor(lds / n) (rounded down to 256 bytes) fit and n + 1
    // do not, as long as lds / (n (n + 1)) exceeds the rounding
    const size_t bytes = (size_t)(lds / n) / 256 * 256;
    if ((size_t)lds / ((size_t)n * (n + 1)) <= 256 || bytes > (size_t)per_block) return 0;
    return bytes;
}

namespace {

// max |cur - prev| over the entries finite in both, and the count of
// entries of cur that are NaN or infinite: per-thread partials, a wave
// butterfly, one atomic per wave (the outputs start at 0; max on the bits
// of non-negative floats orders them as the floats).
__global__ __launch_bounds__(kBlock) void message_stats_kernel(const v4f* cur, const v4f* prev, size_t n4,
                                                               float* max_change, int* non_finite) {
    float mx = 0.0f;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock) {
        const v4f a = cur[i];
        const v4f b = prev ? prev[i] : a;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float x = a[k], y = b[k];
            if (!__builtin_isfinite(x)) ++bad;
            else if (__builtin_isfinite(y)) mx = fmaxf(mx, fabsf(x - y));
        }
    }
#pragma unroll
    for (int w = 32; w >= 1; w /= 2) {
        mx = fmaxf(mx, __shfl_xor(mx, w));
        bad += __shfl_xor(bad, w);
    }
    if ((threadIdx.x & 63) == 0) {
        if (max_change) atomicMax(reinterpret_cast<unsigned*>(max_change), __float_as_uint(mx));
        if (non_finite && bad) atomicAdd(non_finite, bad);
    }
}

__global__ void zero_kernel(unsigned* a, unsigned* b) {
    if (threadIdx.x == 0) {
        if (a) *a = 0u;
        if (b) *b = 0u;
    }
}

}  // namespace

hipError_t launch_message_stats(const float* cur, const float* prev, size_t n, float* max_change, int* non_finite,
                                hipStream_t s) {
    // zeroed by a kernel, not hipMemsetAsync: the call may be captured in a graph
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(max_change),
                       reinterpret_cast<unsigned*>(non_finite));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n4 = n / 4;
    const int cus = cu_count();
    const size_t want = (n4 + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(want, (size_t)(cus > 0 ? cus : 256) * 8));
    hipLaunchKernelGGL(message_stats_kernel, dim3(blocks), dim3(kBlock), 0, s, reinterpret_cast<const v4f*>(cur),
                       reinterpret_cast<const v4f*>(prev), n4, max_change, non_finite);
    return hipGetLastError();
}

int lds_blocks_per_cu(size_t bytes) {
    int dev = 0, per_cu = 0, per_block = 0;
    if (bytes == 0 || hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    if (bytes > (size_t)per_block) return 0;
    return (int)((size_t)per_cu / bytes);
}

int cu_count() {
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cus[kMaxDevices];  // 0: not yet queried
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 0;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

size_t dense_lds_need(int M, int mode) {
    if (mode == kSum && M == 32) return dense_mfma_lds_bytes<8>();
    if (mode == kSum && M == 64) return dense_mfma_lds_bytes<16>();
    return dense_lds_bytes(lanes_for(M), M, mode);
}

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
    if (n % 4 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0) {
        size_t blocks = (n / 4 + kBlock - 1) / kBlock;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(fill4_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, reinterpret_cast<v4f*>(dst),
                           n / 4, value);
        return hipGetLastError();
    }
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_validate_unary(const float* g, int N, int M, int* flag, hipStream_t stream) {
    hipError_t e = launch_fill(reinterpret_cast<float*>(flag), 1, 0.0f, stream);  // int 0
    if (e != hipSuccess || N <= 0) return e;
    hipLaunchKernelGGL(validate_unary_kernel, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, g,
                       N, M, flag);
    return hipGetLastError();
}

hipError_t launch_fill_border(float* msg, int H, int W, int M, float value, hipStream_t stream) {
    const size_t n = (size_t)2 * (H + W) * M;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_border_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, msg,
                       H, W, M, value);
    return hipGetLastError();
}

}  // namespace bpk
