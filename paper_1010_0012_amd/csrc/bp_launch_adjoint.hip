// Instantiation and dispatch of the adjoint kernels.
#include "bp_adjoint.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

// Fixed-order sum of the per-workgroup partials into out[0] (one workgroup).
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const float* part, int n, float* out) {
    __shared__ float s[kBlock];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += kBlock) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w /= 2) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}


// Register-window widths compiled for the adjoint (sum-product only); the
// window reaches K*LPL labels each side and must fit the kAdjTab tables.
template <int LPL> struct AdjK;
template <> struct AdjK<1> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 15}; };
template <> struct AdjK<2> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8}; };
template <> struct AdjK<4> { static constexpr int v[] = {0, 1, 2, 3, 4}; };
template <> struct AdjK<8> { static constexpr int v[] = {0, 1, 2}; };

template <int LPL>
int adj_round_k(int k) {
    for (int c : AdjK<LPL>::v)
        if (c >= k && c * LPL < kAdjTab) return c;
    return -1;
}

template <int LPL, int K>
hipError_t go_step(const AdjointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((adjoint_step_kernel<LPL, K>), dim3(adjoint_blocks(a.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int LPL>
hipError_t step_k(const AdjointArgs& a, int T, hipStream_t s) {
    switch (adj_round_k<LPL>(window_lanes(T, LPL))) {
        case 0: return go_step<LPL, 0>(a, s);
        case 1: return go_step<LPL, 1>(a, s);
        case 2: return go_step<LPL, 2>(a, s);
        case 3: if constexpr (LPL <= 4) return go_step<LPL, 3>(a, s); break;
        case 4: if constexpr (LPL <= 4) return go_step<LPL, 4>(a, s); break;
        case 6: if constexpr (LPL <= 2) return go_step<LPL, 6>(a, s); break;
        case 8: if constexpr (LPL <= 2) return go_step<LPL, 8>(a, s); break;
        case 15: if constexpr (LPL == 1) return go_step<LPL, 15>(a, s); break;
        default: break;
    }
    return hipErrorInvalidValue;
}

template <int LPL>
hipError_t go_seed(const SeedArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((adjoint_seed_kernel<LPL>), dim3(adjoint_blocks(a.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

unsigned adjoint_blocks(int N) { return (unsigned)((N + kBlock / kRow - 1) / (kBlock / kRow)); }

bool adjoint_supported(int M, int T) {
    switch (pick_lpl(M)) {
        case 1: return adj_round_k<1>(window_lanes(T, 1)) >= 0;
        case 2: return adj_round_k<2>(window_lanes(T, 2)) >= 0;
        case 4: return adj_round_k<4>(window_lanes(T, 4)) >= 0;
        case 8: return adj_round_k<8>(window_lanes(T, 8)) >= 0;
        default: return false;
    }
}

hipError_t launch_adjoint_step(const AdjointArgs& a, int T, hipStream_t stream) {
    switch (pick_lpl(a.M)) {
        case 1: return step_k<1>(a, T, stream);
        case 2: return step_k<2>(a, T, stream);
        case 4: return step_k<4>(a, T, stream);
        case 8: return step_k<8>(a, T, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_seed(const SeedArgs& a, hipStream_t stream) {
    switch (pick_lpl(a.M)) {
        case 1: return go_seed<1>(a, stream);
        case 2: return go_seed<2>(a, stream);
        case 4: return go_seed<4>(a, stream);
        case 8: return go_seed<8>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sum_partials(const float* part, int n, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, stream, part, n, out);
    return hipGetLastError();
}

}  // namespace bpk
