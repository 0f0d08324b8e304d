// General sparse-compatible potentials (Sec. 4): up to kMaxTypes potential
// types, each given by its compatible pairs and its constant fbar, assigned
// per edge; the compatibility structure is arbitrary (a per-node
// neighbourhood, a potential that is not a function of x_i - x_j, Sec. 7).
//
// For each type and orientation the tables hold, per target label y, the
// list of compatible sender labels x with f(x, y) (float32) and
// w = f(x, y) - fbar (double), as CSR rows, plus a bitmask of the lists.
//   sum (Eq. 7):  u(y) = fbar * S + sum over the list of w * h(x)
//   max (Eq. 11): u(y) = max(fbar * max h, max over the list of f * h(x)),
//                 exact when every listed f >= fbar;
//   max (Eq. 10): u(y) = max(max over the list of f * h(x),
//                            fbar * max over x outside the list of h(x)),
//                 for types with a listed f < fbar.
// Eq. 10's complement maximum comes from the K largest entries of h (value
// descending, label ascending) with K = longest list + 1: the first of them
// outside list(y) is the maximum over the complement.  Beyond kTopMax the
// complement is scanned label by label against the bitmask.
#pragma once

#include "bp_kernels.hpp"
#include "bp_sweep.hpp"

namespace bpk {

constexpr int kMaxTypes = 16;
constexpr int kTopMax = 32;

struct GenArgs {
    UpdateArgs u;               // grid, buffers, schedule (its tables are unused)
    const unsigned char* type_h;  // [H][W-1] edge types of horizontal pairs, or null (type 0)
    const unsigned char* type_v;  // [H-1][W] edge types of vertical pairs, or null (type 0)
    const int* ptr;             // [n_types * 2][M + 1]: CSR row starts (absolute entry index)
    const int* ent_x;           // sender label of each entry
    const float* ent_f;         // f(x, y) of each entry
    const double* ent_w;        // f(x, y) - fbar of each entry
    const unsigned* mask;       // [n_types * 2][M][mask_words]: bit x of row y set iff x in list(y)
    int mask_words;
    int n_types;
    int n_entries;              // entries of both orientations (ent_x, ent_f, ent_w lengths)
    int top_k;                  // K of the Eq. 10 types (0: none needs Eq. 10)
    float fbar[kMaxTypes];
    double fbar_d[kMaxTypes];
    int eq10[kMaxTypes];        // 1: some listed f < fbar (max-product uses Eq. 10)
};

// Type of the pair between px and its neighbour in direction o (which
// exists); the host validates the maps, and the clamp keeps every table
// access in bounds whatever the caller's memory holds later.
__device__ __forceinline__ int edge_type(const GenArgs& a, const Pixel& px, int o) {
    const int W = a.u.W;
    int t;
    switch (o) {
        case kRight: t = a.type_h ? a.type_h[px.r * (W - 1) + px.c] : 0; break;
        case kLeft: t = a.type_h ? a.type_h[px.r * (W - 1) + px.c - 1] : 0; break;
        case kDown: t = a.type_v ? a.type_v[px.r * W + px.c] : 0; break;
        default: t = a.type_v ? a.type_v[(px.r - 1) * W + px.c] : 0; break;
    }
    return t < a.n_types ? t : a.n_types - 1;
}

// The tables a kernel reads: the global arrays, or the copy a workgroup
// staged in LDS once (f as float32, the labels' h-row slots as bytes,
// M <= 256).  Staged,
// every entry of a row costs LDS reads instead of dependent global loads;
// sum-product then forms f - fbar as (double)f - fbar_d, the same bits as
// the global double table.
template <bool STAGE>
struct GenView {
    const int* ptr;
    const double* w;
    const float* f;
    const int* x32;
    const unsigned char* x8;
    // the slot of entry e's label in a group's h row (row_slot layout): the
    // staged copy holds the slots themselves
    template <int G>
    __device__ __forceinline__ int slot(int e) const {
        if constexpr (STAGE) return x8[e];
        else return row_slot<G>(x32[e]);
    }
    __device__ __forceinline__ double weight(int e, double fbar_d) const {
        if constexpr (STAGE) return (double)f[e] - fbar_d;
        else return w[e];
    }
};

// LDS bytes of the staged tables: row starts, f, labels (8-byte aligned).
constexpr size_t gen_stage_bytes(int n_types, int M, int n_entries) {
    const size_t ptr = ((size_t)n_types * 2 * (M + 1) * sizeof(int) + 7) / 8 * 8;
    return (ptr + (size_t)n_entries * (sizeof(float) + 1) + 7) / 8 * 8;
}

// Stage the tables into LDS at base (all threads of the workgroup; the
// caller's barrier publishes them), or view the global arrays.
template <bool STAGE, int NT, int G>
__device__ __forceinline__ GenView<STAGE> gen_view(const GenArgs& a, char* base) {
    GenView<STAGE> v;
    if constexpr (STAGE) {
        const int n_ptr = a.n_types * 2 * (a.u.M + 1);
        int* ptr = reinterpret_cast<int*>(base);
        float* f = reinterpret_cast<float*>(base + ((size_t)n_ptr * sizeof(int) + 7) / 8 * 8);
        unsigned char* x8 = reinterpret_cast<unsigned char*>(f + a.n_entries);
        for (int i = threadIdx.x; i < n_ptr; i += NT) ptr[i] = a.ptr[i];
        for (int e = threadIdx.x; e < a.n_entries; e += NT) {
            f[e] = a.ent_f[e];
            x8[e] = (unsigned char)row_slot<G>(a.ent_x[e]);
        }
        v.ptr = ptr;
        v.w = nullptr;
        v.f = f;
        v.x8 = x8;
        v.x32 = nullptr;
    } else {
        v.ptr = a.ptr;
        v.w = a.ent_w;
        v.f = a.ent_f;
        v.x32 = a.ent_x;
        v.x8 = nullptr;
    }
    return v;
}

constexpr size_t general_lds_bytes(int G) {
    // per group: h (4G doubles), the top values (kTopMax doubles) and labels (kTopMax ints)
    return (size_t)(kBlock / G) * (G * kLpl * sizeof(double) + kTopMax * (sizeof(double) + sizeof(int)));
}

// CSR table slot of edge type k for messages travelling towards o: the
// tables are stored per orientation (towards right/down, towards left/up).
__device__ __forceinline__ int table_slot(int k, int o) { return 2 * k + ((o == kRight || o == kDown) ? 0 : 1); }

// One message of edge type k towards o from this lane's h (Eq. 7 for sum;
// Eq. 11, or Eq. 10 where the type needs it, for max), normalised into m.
// hs, top_v, top_i: this group's LDS rows, shared only by the group's lanes
// (one wave), so wave-level ordering suffices and groups need not call it
// together.
template <int G, int MODE, bool EQ10, bool STAGE>
__device__ __forceinline__ void general_message(const GenArgs& a, const GenView<STAGE>& v, int k, int o,
                                                const double (&h)[kLpl], double* hs, double* top_v, int* top_i,
                                                int pos, float (&m)[kLpl]) {
    const int M = a.u.M;
    const int x0 = pos * kLpl;
    const bool full = M == G * kLpl;
    wave_sync();  // the previous message is done with hs and the top list
#pragma unroll
    for (int i = 0; i < kLpl; ++i) hs[i * G + pos] = h[i];  // row_slot layout
    const int ts = table_slot(k, o);
    const int* pt = v.ptr + ts * (M + 1);
    double u[kLpl];
    if constexpr (MODE == kSum) {
        wave_sync();
        const double base = a.fbar_d[k] * group_sum_d<G>((h[0] + h[1]) + (h[2] + h[3]));
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            const int y = x0 + i;
            double acc = base;
            if (y < M)
                for (int e = pt[y]; e < pt[y + 1]; ++e)
                    acc = fma(v.weight(e, a.fbar_d[k]), hs[v.template slot<G>(e)], acc);
            u[i] = acc;
        }
    } else {
        const double hm = group_max_d<G>(fmax(fmax(h[0], h[1]), fmax(h[2], h[3])));
        const bool topk = EQ10 && a.top_k <= kTopMax;
        if (topk) group_top_k<G>(h, M, x0, pos, a.top_k, top_v, top_i);  // the top_k largest entries of h
        wave_sync();
        const double fb = (double)a.fbar[k];
        const unsigned* mrow = a.mask + (size_t)ts * M * a.mask_words;
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            const int y = x0 + i;
            double inside = 0.0;
            if (y < M)
                for (int e = pt[y]; e < pt[y + 1]; ++e)
                    inside = fmax(inside, (double)v.f[e] * hs[v.template slot<G>(e)]);
            double outside;
            if (!EQ10 || !a.eq10[k]) {
                outside = fb * hm;  // Eq. 11: f >= fbar on the list
            } else if (y >= M) {
                outside = 0.0;
            } else {
                // Eq. 10: fbar times the largest h outside list(y) (0 if the list is everything)
                const unsigned* row = mrow + (size_t)y * a.mask_words;
                double c = 0.0;
                if (topk) {
                    for (int r = 0; r < a.top_k; ++r) {
                        const int x = top_i[r];
                        if (x >= M) break;
                        if (!((row[x >> 5] >> (x & 31)) & 1u)) { c = top_v[r]; break; }
                    }
                } else {
                    for (int x = 0; x < M; ++x)
                        if (!((row[x >> 5] >> (x & 31)) & 1u)) c = fmax(c, hs[row_slot<G>(x)]);
                }
                outside = fb * c;
            }
            u[i] = fmax(inside, outside);
        }
    }
    normalise_d<G>(u, M, x0, full, m);
}

// LDS rows of one group: h, then (per group) the top values and labels.
template <int G>
__device__ __forceinline__ void general_lds_rows(double* lds_d, int groups, int grp, double*& hs, double*& top_v,
                                                 int*& top_i) {
    constexpr int CAP = G * kLpl;
    hs = lds_d + grp * CAP;
    top_v = lds_d + groups * CAP + grp * kTopMax;
    top_i = reinterpret_cast<int*>(lds_d + groups * CAP + groups * kTopMax) + grp * kTopMax;
}

// One tile of kBlock/G pixels per workgroup, or (PERSIST) a grid of
// resident workgroups that each stage the tables once and stride over the
// tiles: staging per tile costs one table copy per 16 pixels at M = 64
// (for four types, about 440 MB of L2-to-LDS traffic per iteration beside
// the 707 MB the update itself moves), while the loop costs about ten
// registers (a wave per SIMD); the host takes PERSIST for large tables.
template <int G, int MODE, bool EQ10, bool STAGE, bool PERSIST>
__global__ __launch_bounds__(kBlock) void general_update_kernel(GenArgs a, int stage_bytes) {
    extern __shared__ double lds_d[];
    const GenView<STAGE> v = gen_view<STAGE, kBlock, G>(a, reinterpret_cast<char*>(lds_d));
    if constexpr (STAGE) __syncthreads();
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int M = a.u.M;
    const int x0 = pos * kLpl;
    const bool full = M == G * kLpl;
    double* hs;
    double* top_v;
    int* top_i;
    general_lds_rows<G>(lds_d + stage_bytes / sizeof(double), RPB, grp, hs, top_v, top_i);
    const size_t plane = (size_t)a.u.N * M;
    auto run_tile = [&](int tile) {
        const Pixel px = map_slot(tile * RPB + grp, a.u);
        PixelInputs in;
        if (px.ok) load_pixel(a.u, px, x0, full, in); else dummy_pixel(in);
        double h[4][kLpl];
        make_h_d(in, h);
        // unrolled: indexed by a loop counter, h[o] and px.has[o] would live
        // in scratch memory
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const bool live = px.ok && px.has[o];
            const int k = live ? edge_type(a, px, o) : 0;
            float m[kLpl];
            general_message<G, MODE, EQ10, STAGE>(a, v, k, o, h[o], hs, top_v, top_i, pos, m);
            store_message(a.u.out, plane, M, a.u.W, px, o, x0, full, m);
        }
    };
    if constexpr (PERSIST) {
        const int n_tiles = (a.u.n_slots + RPB - 1) / RPB;
        for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) run_tile(tile);
    } else {
        run_tile((int)blockIdx.x);
    }
}

// One directional pass of the sweep schedule (Sec. 6) with general
// potentials or Eq. 10 (a.u.dir = direction the messages travel, in place):
// the scanline walk of sweep_pass_kernel with general_message per step.
constexpr size_t general_sweep_lds_bytes(int G) {
    return (size_t)(kSweepBlock / G) * (G * kLpl * sizeof(double) + kTopMax * (sizeof(double) + sizeof(int)));
}

template <int G, int MODE, bool EQ10, bool STAGE>
__global__ __launch_bounds__(kSweepBlock) void general_sweep_kernel(GenArgs a, int stage_bytes) {
    extern __shared__ double lds_d[];
    const GenView<STAGE> v = gen_view<STAGE, kSweepBlock, G>(a, reinterpret_cast<char*>(lds_d));
    if constexpr (STAGE) __syncthreads();
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    double* hs;
    double* top_v;
    int* top_i;
    general_lds_rows<G>(lds_d + stage_bytes / sizeof(double), kSweepBlock / G, grp, hs, top_v, top_i);
    int blk, dir0;
    sweep_block_dir(a.u, blk, dir0);
    const bool horiz = dir0 == kLeft || dir0 == kRight;
    const bool live = blk * (kSweepBlock / G) + grp < (horiz ? a.u.H : a.u.W);
    auto msg = [&](const double (&h)[kLpl], int r, int c, int dir, float (&m)[kLpl]) {
        int k = 0;  // groups past the last scanline pass any valid type
        if (live) {
            Pixel px;
            px.r = r;
            px.c = c;
            k = edge_type(a, px, dir);  // the sender always has a neighbour towards dir
        }
        general_message<G, MODE, EQ10, STAGE>(a, v, k, dir, h, hs, top_v, top_i, pos, m);
    };
    if (a.u.M == G * kLpl) sweep_walk<G, true, double>(a.u, msg);
    else sweep_walk<G, false, double>(a.u, msg);
}

}  // namespace bpk
