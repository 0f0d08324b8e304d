// Many independent grid MRFs (uneven H x W, M, T, alpha) updated by one
// persistent launch per iteration.
//
// The host builds, in caller-owned device memory, one descriptor per
// instance and a work queue of items (instance, first pixel, passes of
// kBlock/G pixels), longest first.  Each workgroup walks the queue with a fixed
// stride, so the schedule needs no atomics and nothing to reset between
// graph replays; every item is an independent piece of the same
// synchronous update, so the result does not depend on which workgroup
// runs it.  A switch on the instance's code path selects the compiled
// (lanes per pixel, window width) variant of the update.
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

constexpr int kBatchTab = 16;      // window taps per instance table (TW <= 8 used)

// Code paths of the batched update: (lanes per pixel G, window half-width
// TW), one persistent kernel each; an instance with truncation T runs the
// smallest TW >= T for its G, the same choice as a single-grid update.  Every
// M <= 256 and T <= 8 has a path.
constexpr int kBatchClasses = 5;   // G = 4, 8, 16, 32, 64
constexpr int kBatchTws = 7;       // TW = 0, 1, 2, 3, 4, 6, 8
constexpr int kBatchArms = kBatchClasses * kBatchTws;
constexpr int kTwOf[kBatchTws] = {0, 1, 2, 3, 4, 6, 8};
constexpr int arm_g(int a) { return 4 << (a / kBatchTws); }
constexpr int arm_tw(int a) { return kTwOf[a % kBatchTws]; }

struct InstDesc {
    const float* g;          // unary [H][W][M]
    float* msg[2];           // ping-pong inbox planes [4][H][W][M]
    long long belief_off;    // offset of this instance in a concatenated beliefs array
    long long label_off;     // offset in a concatenated labels array
    int H, W, M, N, T;
    int arm;                 // code path: G = arm_g(arm), TW = arm_tw(arm)
    float fbar;              // float32 (max-product)
    float tab_f[kBatchTab];  // f(d), |d| <= T (max-product, float32)
    float tab_wf[kBatchTab]; // f(d) - fbar, |d| <= T (sum-product in float32 arithmetic)
    double fbar_d;           // double (sum-product)
    double tab_wd[kBatchTab];  // f(d) - fbar, |d| <= T (sum-product, double)
};

// One launch of a code path: up to kLaunchInst instances, their descriptors
// passed by value in the kernel arguments (no dependent loads before a
// workgroup's first message load).  Workgroup b serves the instance k whose
// block range [blocks_end[k-1], blocks_end[k]) holds b, covering `passes`
// passes of kBlock/G pixels from (b - blocks_end[k-1]) * passes * kBlock/G.
//
// Two-iteration launches whose instances all have M = 4G and inbox planes
// below 2^32 bytes also carry the row-block layout of
// batch_update2_rows_kernel: instance k gets gxp[k] * H workgroups, gx[k] of
// kBlock/G pixels per grid row padded to gxp[k], a multiple of the XCD
// count, so every instance starts on XCD 0 and each XCD holds one contiguous
// strip of columns in every row (as in the single-grid row-block launch).
constexpr int kLaunchInst = 8;
struct BatchLaunch {
    int n_inst;
    int passes;
    int blocks_end[kLaunchInst];  // inclusive prefix sums of workgroups per instance
    int rows;                     // 1: the row-block layout below is valid
    int rows_end[kLaunchInst];    // inclusive prefix sums of gxp[k] * H
    int gx[kLaunchInst];
    int gxp[kLaunchInst];
    InstDesc inst[kLaunchInst];
};

__device__ __forceinline__ int launch_instance(const BatchLaunch& L, int b) {
    int k = 0;
    while (k + 1 < L.n_inst && b >= L.blocks_end[k]) ++k;  // uniform over the workgroup
    return k;
}

template <int G, int TW, int MODE>
__device__ __forceinline__ void batch_item(const InstDesc& d, int first, int passes, int parity) {
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const float* in = d.msg[parity];
    float* out = d.msg[parity ^ 1];
    const int M = d.M, W = d.W;
    const size_t plane = (size_t)d.N * M;
    const bool full = M == G * kLpl;
    const int x0 = pos * kLpl;
    for (int pass = 0; pass < passes; ++pass) {
        const Pixel px = sync_pixel(first + pass * RPB + grp, d.H, W, d.N);
        if (!px.ok) continue;  // whole groups only
        PixelInputs pin;
        load_pixel_ptr(d.g, in, plane, M, px, x0, full, pin);
        if constexpr (MODE == kSumF32) {
            float h[4][kLpl];
            make_h(pin, h);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float u[kLpl];
                sum_message_f<G, TW>(h[o], d.tab_wf, d.fbar, pos, M, x0, full, u);
                store_message(out, plane, M, W, px, o, x0, full, u);
            }
        } else {
            double h[4][kLpl];
            make_h_d(pin, h);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float u[kLpl];
                if constexpr (MODE == kSum) sum_message_d<G, TW>(h[o], d.tab_wd, d.fbar_d, pos, M, x0, full, u);
                else max_message_d<G, TW>(h[o], d.tab_f, d.fbar, pos, M, x0, full, u);
                store_message(out, plane, M, W, px, o, x0, full, u);
            }
        }
    }
}

// PERSIST: the grid strides over the launch's workgroups and each covers
// L.passes passes; otherwise (one pass per workgroup, one workgroup per
// range) the kernel has no loops and the register budget of the single-grid
// update.
template <int MODE, int G, int TW, bool PERSIST>
__global__ __launch_bounds__(kBlock) void batch_update_kernel(const BatchLaunch L, int parity) {
    if constexpr (PERSIST) {
        const int total = L.blocks_end[L.n_inst - 1];
        for (int b = blockIdx.x; b < total; b += gridDim.x) {
            const int k = launch_instance(L, b);
            const int b0 = k ? L.blocks_end[k - 1] : 0;
            batch_item<G, TW, MODE>(L.inst[k], (b - b0) * (kBlock / G) * L.passes, L.passes, parity);
        }
    } else {
        const int b = blockIdx.x;
        const int k = launch_instance(L, b);
        const int b0 = k ? L.blocks_end[k - 1] : 0;
        batch_item<G, TW, MODE>(L.inst[k], (b - b0) * (kBlock / G), 1, parity);
    }
}

// Two synchronous iterations per launch (the per-pixel work of
// sparse_update2_kernel) over the launch's instances, msg[parity] ->
// msg[parity ^ 1]; FULL: every instance of the launch has M = 4G.
template <int MODE, int G, int TW, bool FULL>
__global__ __launch_bounds__(kBlock) void batch_update2_kernel(const BatchLaunch L, int parity) {
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int total = L.blocks_end[L.n_inst - 1];
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int k = launch_instance(L, b);
        const InstDesc& d = L.inst[k];
        const int first = (b - (k ? L.blocks_end[k - 1] : 0)) * RPB * L.passes;
        for (int pass = 0; pass < L.passes; ++pass) {
            const Pixel px = sync_pixel(first + pass * RPB + grp, d.H, d.W, d.N);
            if (!px.ok) continue;  // whole groups only
            pair_pixel<G, TW, MODE, FULL>(d.g, d.msg[parity], d.msg[parity ^ 1], nullptr, d.H, d.W, d.M, px, pos,
                                          d.tab_wd, d.fbar_d, MODE == kSumF32 ? d.tab_wf : d.tab_f, d.fbar);
        }
    }
}

// The row-block form of batch_update2_kernel (L.rows set; one workgroup per
// range, grid = L.rows_end[n_inst - 1]): the per-pixel code of the
// single-grid row-block launch, so each instance's result equals its
// single-grid pair launch bit for bit.
template <int MODE, int G, int TW>
__global__ __launch_bounds__(kBlock) void batch_update2_rows_kernel(const BatchLaunch L, int parity) {
    constexpr int PPB = kBlock / G;
    const int b = (int)blockIdx.x;
    int k = 0;
    while (k + 1 < L.n_inst && b >= L.rows_end[k]) ++k;  // uniform over the workgroup
    const InstDesc& d = L.inst[k];
    // XCD x (workgroup b runs on XCD b mod 8, and every instance's range
    // starts at a multiple of 8) holds the contiguous column blocks
    // [x gxp/8, (x+1) gxp/8) of every row of the instance
    const int lb = b - (k ? L.rows_end[k - 1] : 0);
    const int wide = L.gxp[k] / kXcds;
    const int kx = lb / kXcds;
    const int r = kx / wide;
    const int cb = (lb % kXcds) * wide + (kx - r * wide);
    if (cb >= L.gx[k]) return;  // padding: whole workgroup
    const int c = cb * PPB + (int)(threadIdx.x / G);
    if (c >= d.W) return;  // whole groups only
    pair_rows_pixel<G, TW, MODE>(d.g, d.msg[parity], d.msg[parity ^ 1], nullptr, d.H, d.W, r, c,
                                 (int)(threadIdx.x & (G - 1)), d.tab_wd, d.fbar_d,
                                 MODE == kSumF32 ? d.tab_wf : d.tab_f, d.fbar);
}

// Beliefs (Eq. 3) and MAP labels of every instance into concatenated outputs.
template <int G>
__global__ __launch_bounds__(kBlock) void batch_readout_kernel(const BatchLaunch L, int parity, float* beliefs,
                                                               int* labels) {
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int x0 = pos * kLpl;
    const int total = L.blocks_end[L.n_inst - 1];
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int k = launch_instance(L, b);
        const InstDesc& d = L.inst[k];
        const int first = (b - (k ? L.blocks_end[k - 1] : 0)) * RPB * L.passes;
        const size_t plane = (size_t)d.N * d.M;
        const bool full = d.M == G * kLpl;
        for (int pass = 0; pass < L.passes; ++pass) {
            const Pixel px = sync_pixel(first + pass * RPB + grp, d.H, d.W, d.N);
            if (!px.ok) continue;
            PixelInputs pin;
            load_pixel_ptr(d.g, d.msg[parity], plane, d.M, px, x0, full, pin);
            readout_pixel<G>(pin, d.M, x0, full, beliefs ? beliefs + d.belief_off + (size_t)px.p * d.M : nullptr,
                             labels ? labels + d.label_off + px.p : nullptr);
        }
    }
}

}  // namespace bpk
