// Instantiation and dispatch of the adjoint kernels.
#include "bp_adjoint.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

template <int G>
unsigned adjoint_blocks_g(int N) { return (unsigned)((N + kBlock / G - 1) / (kBlock / G)); }

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


// Window half-widths compiled for the adjoint (sum-product only); every tap
// index must fit the kAdjTab tables and the window must stay in the group.
template <int G> struct AdjTw { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 12, 16}; };
template <> struct AdjTw<4> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 12}; };

template <int G>
int adj_round_tw(int T) {
    for (int c : AdjTw<G>::v)
        if (c >= T && c < kAdjTab) return c;
    return -1;
}

template <int G, int TW>
hipError_t go_step(const AdjointArgs& a, hipStream_t s) {
    if (a.M == G * kLpl)
        hipLaunchKernelGGL((adjoint_step_kernel<G, TW, true>), dim3(adjoint_blocks_g<G>(a.N)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((adjoint_step_kernel<G, TW, false>), dim3(adjoint_blocks_g<G>(a.N)), dim3(kBlock), 0, s,
                           a);
    return hipGetLastError();
}

template <int G, int I = 0>
hipError_t step_tw(const AdjointArgs& a, int tw, hipStream_t s) {
    constexpr int n = sizeof(AdjTw<G>::v) / sizeof(int);
    if constexpr (I < n) {
        constexpr int TW = AdjTw<G>::v[I];
        if (tw == TW) return go_step<G, TW>(a, s);
        return step_tw<G, I + 1>(a, tw, s);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int G>
hipError_t go_seed(const SeedArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((adjoint_seed_kernel<G>), dim3(adjoint_blocks_g<G>(a.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

unsigned adjoint_blocks(int M, int N) {
    switch (lanes_for(M)) {
        case 4: return adjoint_blocks_g<4>(N);
        case 8: return adjoint_blocks_g<8>(N);
        case 16: return adjoint_blocks_g<16>(N);
        case 32: return adjoint_blocks_g<32>(N);
        default: return adjoint_blocks_g<64>(N);
    }
}

bool adjoint_supported(int M, int T) {
    switch (lanes_for(M)) {
        case 4: return adj_round_tw<4>(T) >= 0;
        case 8: return adj_round_tw<8>(T) >= 0;
        case 16: return adj_round_tw<16>(T) >= 0;
        case 32: return adj_round_tw<32>(T) >= 0;
        case 64: return adj_round_tw<64>(T) >= 0;
        default: return false;
    }
}

hipError_t launch_adjoint_step(const AdjointArgs& a, int T, hipStream_t stream) {
    switch (lanes_for(a.M)) {
        case 4: return step_tw<4>(a, adj_round_tw<4>(T), stream);
        case 8: return step_tw<8>(a, adj_round_tw<8>(T), stream);
        case 16: return step_tw<16>(a, adj_round_tw<16>(T), stream);
        case 32: return step_tw<32>(a, adj_round_tw<32>(T), stream);
        case 64: return step_tw<64>(a, adj_round_tw<64>(T), stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_seed(const SeedArgs& a, hipStream_t stream) {
    switch (lanes_for(a.M)) {
        case 4: return go_seed<4>(a, stream);
        case 8: return go_seed<8>(a, stream);
        case 16: return go_seed<16>(a, stream);
        case 32: return go_seed<32>(a, stream);
        case 64: return go_seed<64>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sum_partials(const float* part, int n, float* out, hipStream_t stream) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, stream, part, n, out);
    return hipGetLastError();
}

}  // namespace bpk
