// Two synchronous iterations per launch over two-dimensional pixel tiles
// staged in LDS.
//
// The row-block launch reads seventeen label rows per pixel (its own unary
// and, for each of its four neighbours, that neighbour's unary and three
// inbox rows), five of them unique; the repeats come through L2 and keep
// the texture address and data units about 90% busy.  Here a workgroup
// takes a TR x TC tile.  Each group loads its own pixel's unary and four
// inbox rows once, and the groups share out the four rows of every halo
// pixel (the tile's outside neighbours, TR on each side and TC above and
// below); all of it goes to LDS, one barrier, and every neighbour row the
// two iterations need is read from there: 9 row loads per pixel at TR = 4,
// TC = 4, instead of 17.  The arithmetic is the row-block launch's
// (pair_first, pair_second) on the same rows (rows of missing pixels and
// senders read the row of ones), so the results are the same bits.
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

template <int G>
struct TileShape {
    static constexpr int NPX = kBlock / G;               // pixels per tile
    static constexpr int TR = NPX >= 64 ? 8 : 4;         // tile rows (8 x 8 at M = 16)
    static constexpr int TC = NPX / TR;                  // tile columns
    static constexpr int NH = 2 * (TR + TC);             // halo pixels
    static constexpr int OWN_ROWS = 5 * NPX;             // own pixels: g, inbox L, R, U, D
    static constexpr int HALO_ROWS = 4 * NH;             // halo pixels: the four rows a neighbour's message uses
    static constexpr int HPG = HALO_ROWS / NPX;          // halo rows each group loads
    static constexpr size_t LDS = (size_t)(OWN_ROWS + HALO_ROWS) * 16 * G;
    static_assert(HALO_ROWS % NPX == 0, "halo rows shared evenly among the groups");
};

template <int G>
constexpr size_t tile_lds_bytes() {
    return TileShape<G>::LDS;
}

// Tiles in row-major order per XCD strip: tiles_x tile columns padded to
// txp, a multiple of the XCD count; XCD x holds tile columns [x txp/8,
// (x + 1) txp/8) of every tile row (as the row-block launch's wide strips),
// so the halo rows of the tile row above come through the same L2.  M = 4G,
// synchronous, inbox planes below 2^32 bytes.
template <int G, int TW, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_tile2_kernel(UpdateArgs a, int txp, int tiles_x) {
    using S = TileShape<G>;
    constexpr int M = 4 * G;
    constexpr int lab = 4 * G;  // floats per label row
    extern __shared__ __attribute__((aligned(16))) float tile_lds[];
    const int wide = txp / kXcds;
    const int xcd = (int)blockIdx.x % kXcds, kk = (int)blockIdx.x / kXcds;
    const int ty = kk / wide;
    const int tx = xcd * wide + (kk - ty * wide);
    if (tx >= tiles_x) return;  // padding: whole workgroup
    const int H = a.H, W = a.W;
    const int r0 = ty * S::TR, c0 = tx * S::TC;
    if (r0 >= H) return;  // whole workgroup
    const int pos = (int)threadIdx.x & (G - 1);
    const int x0 = pos * kLpl;
    const int gi = (int)threadIdx.x / G;  // this group's pixel of the tile
    const int tr = gi / S::TC, tc = gi - tr * S::TC;
    const int r = r0 + tr, c = c0 + tc;
    const size_t plane = (size_t)H * W * M;

    // this lane's 16 bytes of a row: the unary (d < 0) or inbox plane d of
    // pixel (pr, pc), or the row of ones where the pixel or that sender is
    // missing
    auto row_ptr = [&](int pr, int pc, int d) -> const float* {
        const bool in = pr >= 0 && pr < H && pc >= 0 && pc < W;
        const bool snd = d < 0 || (d == kLeft && pc > 0) || (d == kRight && pc + 1 < W) || (d == kUp && pr > 0) ||
                         (d == kDown && pr + 1 < H);
        if (!(in && snd)) return kOnesRow.v + x0;
        const size_t off = ((size_t)pr * W + pc) * M + x0;
        return d < 0 ? a.g + off : a.in + d * plane + off;
    };
    auto lds_row = [&](int row) { return tile_lds + (size_t)row * lab + x0; };
    auto put = [&](int row, v4f v) { *reinterpret_cast<v4f*>(lds_row(row)) = v; };

    // Own pixel: the unary and the four inbox rows.
    v4f own[5];
    own[0] = ld(reinterpret_cast<const v4f*>(row_ptr(r, c, -1)), kUnaryNT);
#pragma unroll
    for (int d = 0; d < 4; ++d) own[1 + d] = ld(reinterpret_cast<const v4f*>(row_ptr(r, c, d)), kMsgNT);
    // Halo rows: row hr = gi HPG + j is row i = hr % 4 of halo pixel h = hr / 4;
    // halo pixels run left column, right column, top row, bottom row, and
    // each stores the rows its message into the tile uses, in pair_compute's
    // order {g, the two partial-product rows, the far-side row}.
    v4f halo[S::HPG];
#pragma unroll
    for (int j = 0; j < S::HPG; ++j) {
        const int hr = gi * S::HPG + j;
        const int h = hr >> 2, i = hr & 3;
        int pr, pc, k;  // the halo pixel and its direction from the tile pixel it sends to
        if (h < S::TR) { pr = r0 + h; pc = c0 - 1; k = kLeft; }
        else if (h < 2 * S::TR) { pr = r0 + h - S::TR; pc = c0 + S::TC; k = kRight; }
        else if (h < 2 * S::TR + S::TC) { pr = r0 - 1; pc = c0 + h - 2 * S::TR; k = kUp; }
        else { pr = r0 + S::TR; pc = c0 + h - 2 * S::TR - S::TC; k = kDown; }
        // pair_sources(k): horizontal neighbours use U, D and their own
        // side's row, vertical ones L, R and theirs
        const int ka = (k == kLeft || k == kRight) ? kUp : kLeft;
        const int d = i == 0 ? -1 : i == 1 ? ka : i == 2 ? ka + 1 : k;
        halo[j] = ld(reinterpret_cast<const v4f*>(row_ptr(pr, pc, d)), d < 0 ? kUnaryNT : kMsgNT);
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) put(5 * gi + d, own[d]);
#pragma unroll
    for (int j = 0; j < S::HPG; ++j) put(S::OWN_ROWS + gi * S::HPG + j, halo[j]);
    __syncthreads();

    // The four rows of the neighbour in direction k that its message to
    // this pixel uses: a tile pixel's planes, or a halo pixel's rows.
    float rows[4][4][kLpl];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int src[3];
        pair_sources(k, src);
        int ntr = tr, ntc = tc, h;
        bool inside;
        if (k == kLeft) { ntc = tc - 1; inside = tc > 0; h = tr; }
        else if (k == kRight) { ntc = tc + 1; inside = tc + 1 < S::TC; h = S::TR + tr; }
        else if (k == kUp) { ntr = tr - 1; inside = tr > 0; h = 2 * S::TR + tc; }
        else { ntr = tr + 1; inside = tr + 1 < S::TR; h = 2 * S::TR + S::TC + tc; }
        const int np = ntr * S::TC + ntc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = inside ? 5 * np + (i == 0 ? 0 : 1 + src[i - 1]) : S::OWN_ROWS + 4 * h + i;
            const v4f v = *reinterpret_cast<const v4f*>(lds_row(row));
            rows[k][i][0] = v.x;
            rows[k][i][1] = v.y;
            rows[k][i][2] = v.z;
            rows[k][i][3] = v.w;
        }
    }
    const bool ok = r < H && c < W;
    const bool has[4] = {c > 0, c + 1 < W, r > 0, r + 1 < H};
    float gp[kLpl] = {own[0].x, own[0].y, own[0].z, own[0].w};
    const size_t p_off = ((size_t)r * W + c) * M;
    pair_compute<G, TW, MODE, true>(
        rows, gp, has, pos, M, a.dtab, a.fbar_d, a.tab, a.fbar,
        [&](int k, const float (&m)[kLpl]) {
            if (a.mid && ok && has[k]) store_labels<kMsgNT>(a.mid + k * plane + p_off, x0, M, true, m);
        },
        [&](int o, const float (&u)[kLpl]) {
            if (ok && has[o]) {
                const long q = (long)p_off + (o == kLeft ? -M : o == kRight ? M : o == kUp ? -(long)W * M : (long)W * M);
                store_labels<kMsgNT>(a.out + opposite(o) * plane + q, x0, M, true, u);
            }
        });
}

// The checkerboard pass pair (a.colour = c: the passes of colour 1 - c and
// then c, run by the colour-c pixels, as sparse_update2_rows_kernel runs it)
// over 4 x 2NPX/4 tiles: the NPX colour-c pixels of a tile compute; each
// group loads its pixel's unary and the five rows of one colour-(1 - c)
// pixel of the tile, and the groups share out the four rows of the halo
// pixels next to a colour-c pixel (the tile's edge pixels alternate, so
// half of each side: 2 + 2 + 4 + 4 at M = 64, where a tile is 4 x 8).  9 row loads per computing
// pixel instead of 17; the same rows and arithmetic as the row-block
// launch, so the same bits.
template <int G>
struct TileCbShape {
    static constexpr int NPX = kBlock / G;               // computing pixels per tile
    static constexpr int TR = NPX >= 32 ? 8 : 4;         // tile rows
    static constexpr int TC = 2 * NPX / TR;              // tile columns (even)
    static constexpr int NH = TR + TC;                   // halo pixels next to a computing pixel
    static constexpr int OTHER_ROWS = 5 * NPX;           // the other colour's pixels: g, inbox L, R, U, D
    static constexpr int HALO_ROWS = 4 * NH;
    static constexpr int HPG = HALO_ROWS / NPX;
    static constexpr size_t LDS = (size_t)(OTHER_ROWS + HALO_ROWS) * 16 * G;
    static_assert(HALO_ROWS % NPX == 0, "halo rows shared evenly among the groups");
};

template <int G>
constexpr size_t tile_cb_lds_bytes() {
    return TileCbShape<G>::LDS;
}

template <int G, int TW, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_tile2cb_kernel(UpdateArgs a, int txp, int tiles_x) {
    using S = TileCbShape<G>;
    constexpr int M = 4 * G;
    constexpr int lab = 4 * G;
    constexpr int PR = S::TC / 2;  // computing pixels per tile row
    extern __shared__ __attribute__((aligned(16))) float tile_lds[];
    const int wide = txp / kXcds;
    const int xcd = (int)blockIdx.x % kXcds, kk = (int)blockIdx.x / kXcds;
    const int ty = kk / wide;
    const int tx = xcd * wide + (kk - ty * wide);
    if (tx >= tiles_x) return;  // padding: whole workgroup
    const int H = a.H, W = a.W;
    const int r0 = ty * S::TR, c0 = tx * S::TC;  // c0 even
    if (r0 >= H) return;  // whole workgroup
    const int colour = a.colour;
    const int pos = (int)threadIdx.x & (G - 1);
    const int x0 = pos * kLpl;
    const int gi = (int)threadIdx.x / G;
    // tile row tr holds computing pixels at columns 2k + s(tr) and the other
    // colour at 2k + 1 - s(tr), s(tr) = (colour + r0 + tr) & 1 (c0 is even)
    auto shift = [&](int tr) { return (colour + r0 + tr) & 1; };
    const int tr = gi / PR, kc = gi - tr * PR;
    const int tc = 2 * kc + shift(tr);
    const int r = r0 + tr, c = c0 + tc;
    const size_t plane = (size_t)H * W * M;

    auto row_ptr = [&](int pr, int pc, int d) -> const float* {
        const bool in = pr >= 0 && pr < H && pc >= 0 && pc < W;
        const bool snd = d < 0 || (d == kLeft && pc > 0) || (d == kRight && pc + 1 < W) || (d == kUp && pr > 0) ||
                         (d == kDown && pr + 1 < H);
        if (!(in && snd)) return kOnesRow.v + x0;
        const size_t off = ((size_t)pr * W + pc) * M + x0;
        return d < 0 ? a.g + off : a.in + d * plane + off;
    };
    auto lds_row = [&](int row) { return tile_lds + (size_t)row * lab + x0; };
    auto put = [&](int row, v4f v) { *reinterpret_cast<v4f*>(lds_row(row)) = v; };

    // this group's computing pixel's unary, and the five rows of the
    // other-colour pixel gi (the one in the same tile row at 2 kc + 1 - s)
    const v4f gown = ld(reinterpret_cast<const v4f*>(row_ptr(r, c, -1)), kUnaryNT);
    const int oc = c0 + 2 * kc + 1 - shift(tr);
    v4f other[5];
    other[0] = ld(reinterpret_cast<const v4f*>(row_ptr(r, oc, -1)), kUnaryNT);
#pragma unroll
    for (int d = 0; d < 4; ++d) other[1 + d] = ld(reinterpret_cast<const v4f*>(row_ptr(r, oc, d)), kMsgNT);
    // Halo pixels next to a computing pixel: h < TR/2 the left column's (the
    // tile rows whose column 0 computes), then the right column's, then the
    // top row's (above tile row 0's computing pixels), then the bottom row's.
    v4f halo[S::HPG];
#pragma unroll
    for (int j = 0; j < S::HPG; ++j) {
        const int hr = gi * S::HPG + j;
        const int h = hr >> 2, i = hr & 3;
        int pr, pc, k;
        if (h < S::TR / 2) {  // tile rows t with s(t) = 0: t = 2h + s(0)
            pr = r0 + 2 * h + shift(0); pc = c0 - 1; k = kLeft;
        } else if (h < S::TR) {  // tile rows t with s(t) = 1 (column TC - 1 is odd): t = 2h' + 1 - s(0)
            pr = r0 + 2 * (h - S::TR / 2) + 1 - shift(0); pc = c0 + S::TC; k = kRight;
        } else if (h < S::TR + PR) {
            pr = r0 - 1; pc = c0 + 2 * (h - S::TR) + shift(0); k = kUp;
        } else {
            pr = r0 + S::TR; pc = c0 + 2 * (h - S::TR - PR) + shift(S::TR - 1); k = kDown;
        }
        const int ka = (k == kLeft || k == kRight) ? kUp : kLeft;
        const int d = i == 0 ? -1 : i == 1 ? ka : i == 2 ? ka + 1 : k;
        halo[j] = ld(reinterpret_cast<const v4f*>(row_ptr(pr, pc, d)), d < 0 ? kUnaryNT : kMsgNT);
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) put(5 * gi + d, other[d]);
#pragma unroll
    for (int j = 0; j < S::HPG; ++j) put(S::OTHER_ROWS + gi * S::HPG + j, halo[j]);
    __syncthreads();

    // Neighbours of (tr, tc): the other colour, in the tile (other-colour
    // index tr * PR + (column >> 1)) or in the halo.
    float rows[4][4][kLpl];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int src[3];
        pair_sources(k, src);
        int ntr = tr, ntc = tc, h;
        bool inside;
        if (k == kLeft) { ntc = tc - 1; inside = tc > 0; h = tr >> 1; }
        else if (k == kRight) { ntc = tc + 1; inside = tc + 1 < S::TC; h = S::TR / 2 + (tr >> 1); }
        else if (k == kUp) { ntr = tr - 1; inside = tr > 0; h = S::TR + kc; }
        else { ntr = tr + 1; inside = tr + 1 < S::TR; h = S::TR + PR + kc; }
        const int np = ntr * PR + (ntc >> 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = inside ? 5 * np + (i == 0 ? 0 : 1 + src[i - 1]) : S::OTHER_ROWS + 4 * h + i;
            const v4f v = *reinterpret_cast<const v4f*>(lds_row(row));
            rows[k][i][0] = v.x;
            rows[k][i][1] = v.y;
            rows[k][i][2] = v.z;
            rows[k][i][3] = v.w;
        }
    }
    const bool ok = r < H && c < W;
    const bool has[4] = {c > 0, c + 1 < W, r > 0, r + 1 < H};
    float gp[kLpl] = {gown.x, gown.y, gown.z, gown.w};
    const size_t p_off = ((size_t)r * W + c) * M;
    pair_compute<G, TW, MODE, true>(
        rows, gp, has, pos, M, a.dtab, a.fbar_d, a.tab, a.fbar,
        [&](int k, const float (&m)[kLpl]) {
            if (a.mid && ok && has[k]) store_labels<kMsgNT>(a.mid + k * plane + p_off, x0, M, true, m);
        },
        [&](int o, const float (&u)[kLpl]) {
            if (ok && has[o]) {
                const long q = (long)p_off + (o == kLeft ? -M : o == kRight ? M : o == kUp ? -(long)W * M : (long)W * M);
                store_labels<kMsgNT>(a.out + opposite(o) * plane + q, x0, M, true, u);
            }
        });
}

}  // namespace bpk
