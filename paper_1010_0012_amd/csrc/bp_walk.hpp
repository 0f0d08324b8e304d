// Two synchronous iterations per launch as a column walk through LDS.
//
// The row-block launch reads seventeen label rows per pixel, five of them
// unique: each neighbour's unary and inbox rows come again through L2 for
// every receiver, and the texture address and data units, not HBM, set its
// pace.  Here a workgroup owns a strip of kBlock/G columns and walks a chunk
// of grid rows from top to bottom.  Each grid row's unary and four inbox
// planes, over the strip and one halo pixel on each side, are copied once
// into a ring of LDS slots by direct global-to-LDS loads (no registers held
// while in flight), P rows ahead of the row being computed.  Every message
// of the first iteration is computed once, as in the row-block launch, but
// when its sender's row arrives: the vertical ones from the sender's own
// pixel, the horizontal ones into the strip's pixels from the neighbours
// in the same row.  The second iteration of a row runs one step later, when
// the messages from the row below exist.  Both use pair_first and
// pair_second, the arithmetic of the row-block launch, so the two launches
// give the same bits.
//
// Pacing.  Each wave issues the same memory instructions at every step: NI
// global-to-LDS loads for the row P ahead (rows outside the chunk's halo,
// and rows of missing senders, read the read-only row of ones), then S
// buffer stores (the second iteration's four messages, and with a.mid the
// four first-iteration messages into the pixel; lanes that must not store
// use an offset beyond the buffer's size, which the hardware drops, and the
// first two steps and the prologue store nothing that way).  Vector memory
// operations of a wave complete in issue order, so before computing row j
// a wave waits until at most S + (P - 1)(NI + S) of its operations are
// outstanding: those issued after row j's loads.  A barrier then makes
// every wave's part of the slot visible, and the slot of the previous row,
// which every wave has finished reading, takes the loads for row j + P.
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

static_assert(kBlock == 256, "the column walk assumes four waves per workgroup");

template <int G>
struct WalkShape {
    static constexpr int NP = kBlock / G;                         // strip pixels per grid row
    static constexpr int SP = NP + 2;                             // staged pixels: one halo pixel each side
    static constexpr int RPI = 64 / G;                            // label rows per wave load (64 x 16 bytes)
    static constexpr int ROWS = 5 * SP;                           // staged label rows: unary, 4 inbox planes
    static constexpr int NI = (ROWS + 4 * RPI - 1) / (4 * RPI);  // loads per wave per grid row
    static constexpr int SLOT = 4 * NI * 1024;                    // bytes of one ring slot
};

// Grid rows in flight ahead of the one computed: a ring of three slots, two
// workgroups per CU (72 KB at M = 32 and 64).  Measured at 480 x 640,
// float32 arithmetic: a ring of five (one workgroup per CU), of two (three
// per CU), or rows staged through registers instead of direct loads were
// no faster (M = 64) or slower (M = 32).
constexpr int kWalkRows = 2;

template <int G>
constexpr size_t walk_lds_bytes() {
    return (size_t)(kWalkRows + 1) * WalkShape<G>::SLOT;
}

// s_waitcnt with vmcnt <= n (clamped to the 6-bit field; smaller is only
// stricter) and lgkmcnt 0, expcnt untouched.
template <int N>
__device__ __forceinline__ void walk_wait() {
    constexpr int n = N > 63 ? 63 : N;
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4));
}

// Workgroup barrier without a memory fence: a fence would wait for every
// load in flight, the loads for the rows ahead included.  The empty asm
// statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void walk_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

typedef const void __attribute__((address_space(1)))* walk_gptr;
typedef void __attribute__((address_space(3)))* walk_lptr;

// One lane's 16 bytes of an LDS label row.
__device__ __forceinline__ void walk_read(const char* p, float (&v)[kLpl]) {
    const v4f t = *reinterpret_cast<const v4f*>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}

__device__ __forceinline__ void walk_store(__amdgpu_buffer_rsrc_t r, uint32_t off, const float (&v)[kLpl]) {
    __builtin_amdgcn_raw_buffer_store_b128(v4f{v[0], v[1], v[2], v[3]}, r, off, 0, kMsgNT ? 2 : 0);
}

constexpr uint32_t kWalkDrop = 0x80000000u;  // beyond every plane (the walk takes planes below 2^31 bytes)
constexpr int kWalkRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format

// What a workgroup carries from one grid row to the next: the unary of the
// row whose second iteration comes next, the horizontal messages into it,
// and the downward messages of the two rows above.
struct WalkCarry {
    float g_prev[kLpl], hl_prev[kLpl], hr_prev[kLpl], dn_prev[kLpl], dn_prev2[kLpl];
};

// One step of a walk: row j staged at sl (this lane's 16 bytes of the slot's
// label rows), its first-iteration messages, and with `second` the second
// iteration of row j - 1 and its stores.  Without `second`, `drop` issues
// the same number of stores, all dropped.
template <int G, int TW, int MODE>
__device__ __forceinline__ void walk_step(const UpdateArgs& a, const char* sl, int ip, int c, int j, bool second,
                                          bool drop, uint32_t row_b, const __amdgpu_buffer_rsrc_t (&out_r)[4],
                                          const __amdgpu_buffer_rsrc_t (&mid_r)[4], bool with_mid, WalkCarry& w) {
    using S = WalkShape<G>;
    constexpr int M = 4 * G;
    constexpr uint32_t lab_b = 16u * G;
    const int H = a.H, W = a.W;
    const int pos = (int)threadIdx.x & (G - 1);
    auto at = [&](int pl, int px) { return sl + (pl * S::SP + px) * lab_b; };
    // First iteration: the messages (j, c) sends up and down, and those
    // (j, c - 1) and (j, c + 1) send into (j, c).
    float rows[4][kLpl], gc[kLpl], up[kLpl], dn[kLpl], hl[kLpl], hr[kLpl];
    walk_read(at(0, ip), rows[0]);
    walk_read(at(1 + kLeft, ip), rows[1]);
    walk_read(at(1 + kRight, ip), rows[2]);
    walk_read(at(1 + kDown, ip), rows[3]);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) gc[i] = rows[0][i];
    pair_first<G, TW, MODE>(rows, j < H, pos, M, true, a.dtab, a.fbar_d, a.tab, a.fbar, up);
    walk_read(at(1 + kUp, ip), rows[3]);
    pair_first<G, TW, MODE>(rows, j >= 0, pos, M, true, a.dtab, a.fbar_d, a.tab, a.fbar, dn);
    walk_read(at(0, ip - 1), rows[0]);
    walk_read(at(1 + kUp, ip - 1), rows[1]);
    walk_read(at(1 + kDown, ip - 1), rows[2]);
    walk_read(at(1 + kLeft, ip - 1), rows[3]);
    pair_first<G, TW, MODE>(rows, c > 0, pos, M, true, a.dtab, a.fbar_d, a.tab, a.fbar, hl);
    walk_read(at(0, ip + 1), rows[0]);
    walk_read(at(1 + kUp, ip + 1), rows[1]);
    walk_read(at(1 + kDown, ip + 1), rows[2]);
    walk_read(at(1 + kRight, ip + 1), rows[3]);
    pair_first<G, TW, MODE>(rows, c + 1 < W, pos, M, true, a.dtab, a.fbar_d, a.tab, a.fbar, hr);

    if (second) {
        // Second iteration of p = (j - 1, c).
        const int r = j - 1;
        const bool pok = c < W;
        const bool has[4] = {c > 0, c + 1 < W, r > 0, r + 1 < H};
        const uint32_t voff = (uint32_t)r * row_b + (uint32_t)c * lab_b + (uint32_t)pos * 16;
        PixelInputs mid;
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            mid.g[i] = w.g_prev[i];
            mid.m[kLeft][i] = w.hl_prev[i];
            mid.m[kRight][i] = w.hr_prev[i];
            mid.m[kUp][i] = w.dn_prev2[i];
            mid.m[kDown][i] = up[i];
        }
        if (with_mid) {
#pragma unroll
            for (int q = 0; q < 4; ++q) walk_store(mid_r[q], pok && has[q] ? voff : kWalkDrop, mid.m[q]);
        }
        const uint32_t q_off[4] = {voff - lab_b, voff + lab_b, voff - row_b, voff + row_b};
        pair_second<G, TW, MODE, true>(mid, pos, M, a.dtab, a.fbar_d, a.tab, a.fbar,
                                       [&](int o, const float (&u)[kLpl]) {
                                           walk_store(out_r[opposite(o)], pok && has[o] ? q_off[o] : kWalkDrop, u);
                                       });
    } else if (drop) {
        const float zero[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int o = 0; o < 4; ++o) walk_store(out_r[o], kWalkDrop, zero);
        if (with_mid) {
#pragma unroll
            for (int o = 0; o < 4; ++o) walk_store(mid_r[o], kWalkDrop, zero);
        }
    }
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        w.g_prev[i] = gc[i];
        w.hl_prev[i] = hl[i];
        w.hr_prev[i] = hr[i];
        w.dn_prev2[i] = w.dn_prev[i];
        w.dn_prev[i] = dn[i];
    }
}

// Where a workgroup's walk runs and what each lane stages (shared by both
// staging schemes).
template <int G>
struct WalkSetup {
    using S = WalkShape<G>;
    int r0, r1, c, ip, wave, lane, lo, hi;
    uint32_t row_b, plane_b;
    const char* src[S::NI];  // this lane's 16 bytes of staged row t, grid row 0
    uint32_t need[S::NI];    // conditions on the grid row j (bits as in have())
    const char* ones;
    __amdgpu_buffer_rsrc_t out_r[4], mid_r[4];

    // false: the workgroup has no rows (it exits before any barrier).
    __device__ __forceinline__ bool init(const UpdateArgs& a, int ns, int nc, int rc, int per) {
        constexpr uint32_t lab_b = 16u * G;
        const int L = xcd_band_block((int)blockIdx.x, per);
        if (L >= ns * nc) return false;
        const int chunk = L / ns, strip = L - chunk * ns;
        const int H = a.H, W = a.W;
        r0 = chunk * rc;
        if (r0 >= H) return false;
        r1 = min(H, r0 + rc);
        const int c0 = strip * S::NP;
        lane = (int)threadIdx.x & 63;
        wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
        const int pos = (int)threadIdx.x & (G - 1);
        ip = (int)threadIdx.x / G + 1;
        c = c0 + ip - 1;
        row_b = (uint32_t)W * lab_b;
        plane_b = (uint32_t)H * row_b;
        // Staged row t of this wave covers slot rows (wave NI + t) RPI ..
        // + RPI - 1, 16 bytes per lane in lane order.  need[t]: bit 0 the
        // row is one the chunk reads, bit 1 j > 0 (an inbox from above),
        // bit 2 j + 1 < H (from below), bit 3 never (no such column or
        // sender, or a pad row).
#pragma unroll
        for (int t = 0; t < S::NI; ++t) {
            const int R = (wave * S::NI + t) * S::RPI + lane / G;
            const int pl = R / S::SP;
            const int col = c0 - 1 + (R - pl * S::SP);
            const bool ok =
                R < S::ROWS && col >= 0 && col < W && (pl != 1 || col > 0) && (pl != 2 || col + 1 < W);
            need[t] = 1u | (pl == 3 ? 2u : 0u) | (pl == 4 ? 4u : 0u) | (ok ? 0u : 8u);
            const char* base = pl == 0 ? (const char*)a.g : (const char*)a.in + (size_t)(pl - 1) * plane_b;
            src[t] = base + (ok ? (size_t)col * lab_b : 0) + (size_t)pos * 16;
        }
        ones = (const char*)kOnesRow.v + pos * 16;
        lo = max(r0 - 1, 0);
        hi = min(r1, H - 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            out_r[k] = __builtin_amdgcn_make_buffer_rsrc((char*)a.out + (size_t)k * plane_b, 0, (int)plane_b,
                                                         kWalkRsrcWord3);
            mid_r[k] = __builtin_amdgcn_make_buffer_rsrc(a.mid ? (char*)a.mid + (size_t)k * plane_b : (char*)a.out,
                                                         0, (int)plane_b, kWalkRsrcWord3);
        }
        return true;
    }
    __device__ __forceinline__ uint32_t have(int j, int H) const {
        return (j >= lo && j <= hi ? 1u : 0u) | (j > 0 ? 2u : 0u) | (j + 1 < H ? 4u : 0u);
    }
    // This lane's source of staged row t for grid row j (the row of ones
    // where the row does not exist): one address per t on every path.
    __device__ __forceinline__ const char* source(int t, int j, uint32_t hv) const {
        return (need[t] & ~hv) == 0 ? src[t] + (size_t)max(j, 0) * row_b : ones;
    }
};

// ns strips of kBlock/G columns, nc chunks of rc rows; logical workgroup
// chunk * ns + strip, remapped so that XCD x holds the contiguous logical
// range [x per, (x + 1) per): neighbouring strips of a chunk share an L2 and
// walk down together.  M = 4G, synchronous, inbox planes below 2^31 bytes.
// Staging by direct global-to-LDS loads into a ring of P + 1 slots.
template <int G, int TW, int MODE, int P>
__global__ __launch_bounds__(kBlock) void sparse_walk2_kernel(UpdateArgs a, int ns, int nc, int rc, int per) {
    using S = WalkShape<G>;
    constexpr int D = P + 1;
    extern __shared__ __attribute__((aligned(1024))) char walk_lds[];
    WalkSetup<G> ws;
    if (!ws.init(a, ns, nc, rc, per)) return;  // whole workgroup
    const int pos = (int)threadIdx.x & (G - 1);
    const bool with_mid = a.mid != nullptr;

    auto issue_row = [&](int j, int slot) {
        char* dst = walk_lds + slot * S::SLOT + ws.wave * S::NI * 1024;
        const uint32_t hv = ws.have(j, a.H);
#pragma unroll
        for (int t = 0; t < S::NI; ++t)
            __builtin_amdgcn_global_load_lds((walk_gptr)ws.source(t, j, hv), (walk_lptr)(dst + t * 1024), 16, 0, 0);
    };
    WalkCarry w;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) w.g_prev[i] = w.hl_prev[i] = w.hr_prev[i] = w.dn_prev[i] = w.dn_prev2[i] = 1.0f;
    const float zero[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
    // The compiler barriers keep each step's loads ahead of its stores (a
    // store moved above a load would leave the waits one operation short).
#pragma unroll
    for (int t = 0; t < P; ++t) {
        issue_row(ws.r0 - 1 + t, t);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int o = 0; o < 4; ++o) walk_store(ws.out_r[o], kWalkDrop, zero);
        if (with_mid) {
#pragma unroll
            for (int o = 0; o < 4; ++o) walk_store(ws.mid_r[o], kWalkDrop, zero);
        }
        asm volatile("" ::: "memory");
    }
    const int steps = ws.r1 - ws.r0 + 2;  // rows r0 - 1 .. r1
    for (int k = 0; k < steps; ++k) {
        const int j = ws.r0 - 1 + k;
        if (with_mid) walk_wait<8 + (P - 1) * (S::NI + 8)>();
        else walk_wait<4 + (P - 1) * (S::NI + 4)>();
        walk_barrier();
        issue_row(j + P, (k + P) % D);
        asm volatile("" ::: "memory");
        walk_step<G, TW, MODE>(a, walk_lds + (k % D) * S::SLOT + pos * 16, ws.ip, ws.c, j, k >= 2, true, ws.row_b,
                               ws.out_r, ws.mid_r, with_mid, w);
    }
    __builtin_amdgcn_s_waitcnt(0);  // nothing in flight at exit
}

}  // namespace bpk
