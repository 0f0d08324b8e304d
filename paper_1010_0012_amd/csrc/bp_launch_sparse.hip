// Instantiation and dispatch of the sparse O(mM) update kernels.
#include "bp_kernels.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

// Register-window variants compiled per labels-per-lane; a request rounds
// its K up to the next listed value (extra taps have weight 0).
template <int LPL> struct KList;
template <> struct KList<1> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 15}; };
template <> struct KList<2> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8}; };
template <> struct KList<4> { static constexpr int v[] = {0, 1, 2, 3, 4}; };
template <> struct KList<8> { static constexpr int v[] = {0, 1, 2}; };
template <> struct KList<16> { static constexpr int v[] = {0, 1}; };

template <int LPL>
int round_k(int k) {
    for (int c : KList<LPL>::v)
        if (c >= k) return c;
    return -1;
}

inline unsigned blocks_for(int n_slots) {
    return (unsigned)((n_slots + (kBlock / kRow) - 1) / (kBlock / kRow));
}

#ifndef BP_PIX_PER_ROW
#define BP_PIX_PER_ROW 1
#endif

template <int LPL, int K, int MODE>
hipError_t go(const UpdateArgs& a, hipStream_t s) {
    constexpr int P = LPL <= 4 ? BP_PIX_PER_ROW : 1;
    const unsigned blocks = (unsigned)((a.n_slots + (kBlock / kRow) * P - 1) / ((kBlock / kRow) * P));
    hipLaunchKernelGGL((sparse_update_kernel<LPL, K, MODE, P>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int LPL, int MODE>
hipError_t go_wide(const UpdateArgs& a, hipStream_t s) {
    const size_t lds = ((kBlock / kRow) * kRow * LPL + kMaxTab) * sizeof(float);
    hipLaunchKernelGGL((sparse_update_wide_kernel<LPL, MODE>), dim3(blocks_for(a.n_slots)),
                       dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int LPL, int MODE>
hipError_t dispatch_k(const UpdateArgs& a, hipStream_t s) {
    const int k = round_k<LPL>(window_lanes(a.T, LPL));
    switch (k) {
        case 0: return go<LPL, 0, MODE>(a, s);
        case 1: return go<LPL, 1, MODE>(a, s);
        case 2: return go<LPL, 2, MODE>(a, s);
        case 3: if constexpr (LPL <= 4) return go<LPL, 3, MODE>(a, s); break;
        case 4: if constexpr (LPL <= 4) return go<LPL, 4, MODE>(a, s); break;
        case 6: if constexpr (LPL <= 2) return go<LPL, 6, MODE>(a, s); break;
        case 8: if constexpr (LPL <= 2) return go<LPL, 8, MODE>(a, s); break;
        case 15: if constexpr (LPL == 1) return go<LPL, 15, MODE>(a, s); break;
        default: break;
    }
    return go_wide<LPL, MODE>(a, s);
}

template <int MODE>
hipError_t dispatch_lpl(const UpdateArgs& a, hipStream_t s) {
    switch (pick_lpl(a.M)) {
        case 1: return dispatch_k<1, MODE>(a, s);
        case 2: return dispatch_k<2, MODE>(a, s);
        case 4: return dispatch_k<4, MODE>(a, s);
        case 8: return dispatch_k<8, MODE>(a, s);
        case 16: return dispatch_k<16, MODE>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int sparse_variant_k(int M, int T) {
    const int lpl = pick_lpl(M);
    const int k = window_lanes(T, lpl);
    switch (lpl) {
        case 1: return round_k<1>(k);
        case 2: return round_k<2>(k);
        case 4: return round_k<4>(k);
        case 8: return round_k<8>(k);
        case 16: return round_k<16>(k);
        default: return -1;
    }
}

hipError_t launch_sparse(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    return mode == kSum ? dispatch_lpl<kSum>(a, stream) : dispatch_lpl<kMax>(a, stream);
}

}  // namespace bpk
