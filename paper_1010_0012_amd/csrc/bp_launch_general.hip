// General sparse-potential update: instantiations and dispatch.
#include <algorithm>

#include "bp_general.hpp"
#include "bp_launch.hpp"

namespace bpk {
namespace {

// Tables are staged in LDS when they fit beside the per-group rows within
// this budget per workgroup.
constexpr size_t kGenLdsBudget = 64 * 1024;

// Tables of at least this many staged bytes run the persistent kernel
// (measured at 480x640x64: four types, 23 KB, 492 -> 469 us per iteration;
// one type, 6 KB, 302 -> 338 us, the loop's registers costing a wave).
constexpr size_t kGenPersistBytes = 16 * 1024;

template <int G, int MODE, bool EQ10>
hipError_t go_general(const GenArgs& a, hipStream_t s) {
    const unsigned blocks = (unsigned)((a.u.n_slots + (kBlock / G) - 1) / (kBlock / G));
    const size_t st = gen_stage_bytes(a.n_types, a.u.M, a.n_entries);
    if (st + general_lds_bytes(G) <= kGenLdsBudget) {
        const size_t lds = st + general_lds_bytes(G);
        if (st >= kGenPersistBytes) {
            // persistent: as many workgroups as are resident at once
            auto kern = general_update_kernel<G, MODE, EQ10, true, true>;
            int per_cu = 0;
            const int cus = cu_count();
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds) == hipSuccess &&
                per_cu > 0 && cus > 0) {
                const unsigned grid = std::min(blocks, (unsigned)(cus * per_cu));
                hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, a, (int)st);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((general_update_kernel<G, MODE, EQ10, true, false>), dim3(blocks), dim3(kBlock), lds, s,
                           a, (int)st);
    } else {
        hipLaunchKernelGGL((general_update_kernel<G, MODE, EQ10, false, false>), dim3(blocks), dim3(kBlock),
                           general_lds_bytes(G), s, a, 0);
    }
    return hipGetLastError();
}

template <int MODE, bool EQ10>
hipError_t general_g(const GenArgs& a, hipStream_t s) {
    switch (lanes_for(a.u.M)) {
        case 4: return go_general<4, MODE, EQ10>(a, s);
        case 8: return go_general<8, MODE, EQ10>(a, s);
        case 16: return go_general<16, MODE, EQ10>(a, s);
        case 32: return go_general<32, MODE, EQ10>(a, s);
        case 64: return go_general<64, MODE, EQ10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G, int MODE, bool EQ10>
hipError_t go_general_sweep(const GenArgs& a, hipStream_t s) {
    constexpr int LPB = kSweepBlock / G;
    const int n_lines = (a.u.dir == kLeft || a.u.dir == kRight) ? a.u.H : a.u.W;
    const unsigned blocks = (unsigned)((n_lines + LPB - 1) / LPB) * (a.u.both ? 2 : 1);
    const size_t st = gen_stage_bytes(a.n_types, a.u.M, a.n_entries);
    if (st + general_sweep_lds_bytes(G) <= kGenLdsBudget)
        hipLaunchKernelGGL((general_sweep_kernel<G, MODE, EQ10, true>), dim3(blocks), dim3(kSweepBlock),
                           st + general_sweep_lds_bytes(G), s, a, (int)st);
    else
        hipLaunchKernelGGL((general_sweep_kernel<G, MODE, EQ10, false>), dim3(blocks), dim3(kSweepBlock),
                           general_sweep_lds_bytes(G), s, a, 0);
    return hipGetLastError();
}

template <int MODE, bool EQ10>
hipError_t general_sweep_g(const GenArgs& a, hipStream_t s) {
    switch (lanes_for(a.u.M)) {
        case 4: return go_general_sweep<4, MODE, EQ10>(a, s);
        case 8: return go_general_sweep<8, MODE, EQ10>(a, s);
        case 16: return go_general_sweep<16, MODE, EQ10>(a, s);
        case 32: return go_general_sweep<32, MODE, EQ10>(a, s);
        case 64: return go_general_sweep<64, MODE, EQ10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_general_sweep(const GenArgs& a, int mode, hipStream_t stream) {
    if (mode == kSum) return general_sweep_g<kSum, false>(a, stream);
    return a.top_k > 0 ? general_sweep_g<kMax, true>(a, stream) : general_sweep_g<kMax, false>(a, stream);
}

hipError_t launch_general(const GenArgs& a, int mode, hipStream_t stream) {
    if (a.u.n_slots <= 0) return hipSuccess;
    if (mode == kSum) return general_g<kSum, false>(a, stream);
    return a.top_k > 0 ? general_g<kMax, true>(a, stream) : general_g<kMax, false>(a, stream);
}

}  // namespace bpk
