// Instantiation table and dispatch of the sparse O(mM) update kernels,
// included once per mode (bp_launch_sparse_sum.hip, bp_launch_sparse_max.hip).
#pragma once

#include "bp_kernels.hpp"
#include "bp_launch.hpp"
#include "bp_tile.hpp"
#include "bp_walk.hpp"

#include <algorithm>

namespace bpk {

// Window half-widths TW compiled per group size G; a request with truncation
// T runs the smallest listed TW >= T (extra taps have weight 0).  The window
// reaches ceil(TW/4) lanes each side, fewer than G.  Wider requests use the
// runtime-window kernel.
template <int G> struct TwList { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 12, 16}; };
template <> struct TwList<4> { static constexpr int v[] = {0, 1, 2, 3, 4, 6, 8, 12}; };

template <int G>
int round_tw(int T) {
    for (int c : TwList<G>::v)
        if (c >= T) return c;
    return -1;
}

inline int sparse_tw(int M, int T) {
    switch (lanes_for(M)) {
        case 4: return round_tw<4>(T);
        case 8: return round_tw<8>(T);
        case 16: return round_tw<16>(T);
        case 32: return round_tw<32>(T);
        case 64: return round_tw<64>(T);
        default: return -1;
    }
}

template <int G>
unsigned groups_blocks(int n_slots) {
    return (unsigned)((n_slots + kBlock / G - 1) / (kBlock / G));
}

template <int G, int TW, int MODE>
hipError_t go_sparse(const UpdateArgs& a, hipStream_t s) {
    if constexpr (MODE == kMax) {
        if (a.eq10) {  // Eq. 10: one LDS row per group
            hipLaunchKernelGGL((sparse_update_kernel<G, TW, kMax, true>), dim3(groups_blocks<G>(a.n_slots)),
                               dim3(kBlock), (size_t)(kBlock / G) * eq10_row_doubles(G) * sizeof(double), s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sparse_update_kernel<G, TW, MODE>), dim3(groups_blocks<G>(a.n_slots)), dim3(kBlock), 0,
                       s, a);
    return hipGetLastError();
}

template <int G, int MODE>
hipError_t go_sparse_wide(const UpdateArgs& a, hipStream_t s) {
    if (a.eq10) return hipErrorInvalidValue;  // Eq. 10 beyond the register windows runs the general kernel
    hipLaunchKernelGGL((sparse_update_wide_kernel<G, MODE>), dim3(groups_blocks<G>(a.n_slots)), dim3(kBlock),
                       wide_lds_bytes(G), s, a);
    return hipGetLastError();
}

// The column walk: strips of kBlock/G columns, split into row chunks so
// that the workgroups fill the GPU once (as many as fit at once, given the
// ring's LDS).
template <int G, int TW, int MODE>
hipError_t go_walk(const UpdateArgs& a, hipStream_t s) {
    const size_t lds = walk_lds_bytes<G>();
    const int per_cu = lds_blocks_per_cu(lds);
    const int cus = cu_count();
    if (per_cu < 1 || cus < 1) return hipErrorInvalidValue;
    const int ns = (a.W + kBlock / G - 1) / (kBlock / G);
    int nc = std::max(1, std::min(a.H, cus * per_cu / ns));
    const int rc = (a.H + nc - 1) / nc;
    nc = (a.H + rc - 1) / rc;
    const int64_t total = (int64_t)ns * nc;
    const int64_t per = (total + kXcds - 1) / kXcds;
    if (per * kXcds >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sparse_walk2_kernel<G, TW, MODE, kWalkRows>), dim3((unsigned)(per * kXcds)), dim3(kBlock),
                       lds, s, a, ns, nc, rc, (int)per);
    return hipGetLastError();
}

// The tile launch: TR x TC pixel tiles, tile columns padded to a multiple
// of the XCD count for the wide-strip order.
template <int G, int TW, int MODE>
hipError_t go_tile(const UpdateArgs& a, hipStream_t s) {
    using S = TileShape<G>;
    const int tiles_x = (a.W + S::TC - 1) / S::TC, tiles_y = (a.H + S::TR - 1) / S::TR;
    const int txp = (tiles_x + kXcds - 1) / kXcds * kXcds;
    const int64_t total = (int64_t)txp * tiles_y;
    if (total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sparse_tile2_kernel<G, TW, MODE>), dim3((unsigned)total), dim3(kBlock), tile_lds_bytes<G>(),
                       s, a, txp, tiles_x);
    return hipGetLastError();
}

// The checkerboard pass pair over tiles whose colour-c pixels compute.
template <int G, int TW, int MODE>
hipError_t go_tile_cb(const UpdateArgs& a, hipStream_t s) {
    using S = TileCbShape<G>;
    const int tiles_x = (a.W + S::TC - 1) / S::TC, tiles_y = (a.H + S::TR - 1) / S::TR;
    const int txp = (tiles_x + kXcds - 1) / kXcds * kXcds;
    const int64_t total = (int64_t)txp * tiles_y;
    if (total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sparse_tile2cb_kernel<G, TW, MODE>), dim3((unsigned)total), dim3(kBlock),
                       tile_cb_lds_bytes<G>(), s, a, txp, tiles_x);
    return hipGetLastError();
}

// Two synchronous iterations per launch (register windows only), in the
// mapping a.pair_layout asks for where it applies: row blocks (M = 4G and
// an inbox plane below 2^32 bytes) in XCD column strips, row bands or one
// wide strip per XCD, or
// one group per pixel slot (the grid padded to a multiple of the XCD count
// for its band remap; M = 4G selects the branch-free instance), or the
// column walk (synchronous, M = 32 or 64; elsewhere the wide strips).  All
// mappings run the same per-message code, so they give the same bits.
// a.pair_cap: workgroups per CU allowed through the LDS request (0 none; -1
// the default, 4 for float32 arithmetic, none for double; the walk's ring
// sets its own).
template <int G, int TW, int MODE>
hipError_t go_sparse2(const UpdateArgs& a, hipStream_t s) {
    const bool rows = a.M == G * kLpl && (uint64_t)a.N * a.M * sizeof(float) < (uint64_t(1) << 32);
    const int cap = a.pair_cap >= 0 ? a.pair_cap : (MODE == kSumF32 ? 4 : 0);
    const size_t lds = cap > 0 ? lds_cap_bytes(cap) : 0;
    if constexpr (MODE == kSumF32) {
        if (!rows) return hipErrorInvalidValue;  // float32 arithmetic: row-block launches only
    }
    if constexpr (G <= 32) {
        // the tile launch (synchronous: M = 16 .. 128; checkerboard pairs: M = 32 .. 128)
        if (rows && a.pair_layout == kPairTile && a.colour < 0 && lds_blocks_per_cu(tile_lds_bytes<G>()) >= 1)
            return go_tile<G, TW, MODE>(a, s);
        if constexpr (G >= 8) {
            if (rows && a.pair_layout == kPairTile && a.colour >= 0 && lds_blocks_per_cu(tile_cb_lds_bytes<G>()) >= 1)
                return go_tile_cb<G, TW, MODE>(a, s);
        }
    }
    if constexpr (G == 8 || G == 16) {
        // the walk where it applies and its LDS ring fits the device; else the wide strips
        const bool walk = a.pair_layout == kPairWalk && a.colour < 0 &&
                          (uint64_t)a.N * a.M * sizeof(float) <= (uint64_t(1) << 31);
        if (rows && walk && lds_blocks_per_cu(walk_lds_bytes<G>()) >= 1 && cu_count() >= 1)
            return go_walk<G, TW, MODE>(a, s);
    }
    if (rows && (MODE == kSumF32 || a.pair_layout != kPairSlots)) {
        // row-block launch: kBlock/G pixels (or colour slots) of one row per workgroup
        const int slots = a.colour < 0 ? a.W : a.half_w;
        const int gx = (slots + kBlock / G - 1) / (kBlock / G);
        if (a.pair_layout == kPairBands) {
            const int64_t total = (int64_t)gx * a.H;
            const int per = (int)((total + kXcds - 1) / kXcds);
            if ((int64_t)per * kXcds >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
            hipLaunchKernelGGL((sparse_update2_rows_kernel<G, TW, MODE>), dim3((unsigned)(per * kXcds)), dim3(kBlock),
                               lds, s, a, gx, gx, per);
            return hipGetLastError();
        }
        const int gxp = (gx + kXcds - 1) / kXcds * kXcds;
        const int64_t total = (int64_t)gxp * a.H;
        if (total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((sparse_update2_rows_kernel<G, TW, MODE>), dim3((unsigned)total), dim3(kBlock), lds, s, a,
                           gxp, gx, a.pair_layout == kPairWide || a.pair_layout >= kPairWalk ? -1 : 0);
        return hipGetLastError();
    }
    if constexpr (MODE == kSumF32) {
        return hipErrorInvalidValue;
    } else {
        const int nblk = (int)groups_blocks<G>(a.n_slots);
        const int per = (nblk + kXcds - 1) / kXcds;
        if (a.M == G * kLpl)
            hipLaunchKernelGGL((sparse_update2_kernel<G, TW, MODE, true>), dim3((unsigned)(per * kXcds)), dim3(kBlock),
                               lds, s, a, per);
        else
            hipLaunchKernelGGL((sparse_update2_kernel<G, TW, MODE, false>), dim3((unsigned)(per * kXcds)),
                               dim3(kBlock), lds, s, a, per);
        return hipGetLastError();
    }
}

template <int G, int MODE, int I = 0>
hipError_t dispatch2_tw(const UpdateArgs& a, int tw, hipStream_t s) {
    constexpr int n = sizeof(TwList<G>::v) / sizeof(int);
    if constexpr (I < n) {
        constexpr int TW = TwList<G>::v[I];
        if (tw == TW) return go_sparse2<G, TW, MODE>(a, s);
        return dispatch2_tw<G, MODE, I + 1>(a, tw, s);
    } else {
        return hipErrorInvalidValue;  // no register window: the caller runs single launches
    }
}

template <int MODE>
hipError_t dispatch_sparse2(const UpdateArgs& a, hipStream_t s) {
    const int tw = sparse_tw(a.M, a.T);
    switch (lanes_for(a.M)) {
        case 4: return dispatch2_tw<4, MODE>(a, tw, s);
        case 8: return dispatch2_tw<8, MODE>(a, tw, s);
        case 16: return dispatch2_tw<16, MODE>(a, tw, s);
        case 32: return dispatch2_tw<32, MODE>(a, tw, s);
        case 64: return dispatch2_tw<64, MODE>(a, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template <int G, int MODE, int I = 0>
hipError_t dispatch_tw(const UpdateArgs& a, int tw, hipStream_t s) {
    constexpr int n = sizeof(TwList<G>::v) / sizeof(int);
    if constexpr (I < n) {
        constexpr int TW = TwList<G>::v[I];
        if (tw == TW) return go_sparse<G, TW, MODE>(a, s);
        return dispatch_tw<G, MODE, I + 1>(a, tw, s);
    } else if constexpr (MODE == kSumF32) {
        return hipErrorInvalidValue;  // float32 arithmetic: register windows only
    } else {
        return go_sparse_wide<G, MODE>(a, s);
    }
}

template <int MODE>
hipError_t dispatch_sparse(const UpdateArgs& a, hipStream_t s) {
    const int tw = sparse_tw(a.M, a.T);
    switch (lanes_for(a.M)) {
        case 4: return dispatch_tw<4, MODE>(a, tw, s);
        case 8: return dispatch_tw<8, MODE>(a, tw, s);
        case 16: return dispatch_tw<16, MODE>(a, tw, s);
        case 32: return dispatch_tw<32, MODE>(a, tw, s);
        case 64: return dispatch_tw<64, MODE>(a, tw, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bpk
