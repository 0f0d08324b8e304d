// Many independent grid MRFs (uneven H x W, M, T, alpha) updated by one
// persistent launch per iteration.
//
// The host builds, in caller-owned device memory, one descriptor per
// instance and a work queue of items (instance, first pixel, passes of 16
// pixels), longest first.  Each workgroup walks the queue with a fixed
// stride, so the schedule needs no atomics and nothing to reset between
// graph replays; every item is an independent piece of the same
// synchronous update, so the result does not depend on which workgroup
// runs it.  A switch on the instance's code path selects the compiled
// (labels-per-lane, window width) variant of the update.
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

constexpr int kBatchTab = 16;      // window taps per instance table (K*LPL <= 8 used)

// Code paths compiled into the batched kernel: (labels per lane, window
// lanes each side).  T <= 8 for every M <= 128.
constexpr int kBatchArms = 10;
constexpr int kArmLpl[kBatchArms] = {1, 1, 1, 1, 2, 2, 2, 4, 4, 8};
constexpr int kArmK[kBatchArms] = {1, 2, 4, 8, 1, 2, 4, 1, 2, 1};

struct InstDesc {
    const float* g;          // unary [H][W][M]
    float* msg[2];           // ping-pong inbox planes [4][H][W][M]
    long long belief_off;    // offset of this instance in a concatenated beliefs array
    long long label_off;     // offset in a concatenated labels array
    int H, W, M, N, T;
    int arm;                 // index into kArmLpl / kArmK
    float fbar;
    float tab_w[kBatchTab];  // f(d) - fbar, |d| <= T (sum-product)
    float tab_f[kBatchTab];  // f(d), |d| <= T (max-product)
};

struct Item {
    int inst;
    int first;               // first pixel (row-major) of the item
    int passes;              // passes of 16 pixels (one per 16-lane row group)
    int pad;
};

template <int LPL, int K, int MODE>
__device__ __forceinline__ void batch_item(const InstDesc* __restrict__ d, const Item& item, int parity) {
    constexpr int RPB = kBlock / kRow;
    const int lane = threadIdx.x & (kRow - 1);
    const int row = threadIdx.x / kRow;
    const float* in = d->msg[parity];
    float* out = d->msg[parity ^ 1];
    const int M = d->M, W = d->W;
    const size_t plane = (size_t)d->N * M;
    const bool full = M == kRow * LPL;
    const int x0 = lane * LPL;
    const float* tab = MODE == kSum ? d->tab_w : d->tab_f;
    const float fbar = d->fbar;
    for (int pass = 0; pass < item.passes; ++pass) {
        const Pixel px = sync_pixel(item.first + pass * RPB + row, d->H, W, d->N);
        if (!px.ok) continue;  // whole 16-lane rows only
        PixelInputs<LPL> pin;
        load_pixel_ptr<LPL>(d->g, in, plane, M, px, x0, full, pin);
        float h[4][LPL];
        make_h<LPL>(pin, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[LPL];
            const float s = row_total<LPL, MODE>(h[o]);
            window_apply<LPL, K, MODE>(h[o], tab, fbar * s, u);
            normalise_store_ptr<LPL>(out, plane, M, W, px, o, x0, full, u);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void batch_update_kernel(const InstDesc* __restrict__ inst,
                                                              const Item* __restrict__ items,
                                                              int n_items, int parity) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = items[it];
        const InstDesc* d = inst + item.inst;
        switch (d->arm) {
            case 0: batch_item<1, 1, MODE>(d, item, parity); break;
            case 1: batch_item<1, 2, MODE>(d, item, parity); break;
            case 2: batch_item<1, 4, MODE>(d, item, parity); break;
            case 3: batch_item<1, 8, MODE>(d, item, parity); break;
            case 4: batch_item<2, 1, MODE>(d, item, parity); break;
            case 5: batch_item<2, 2, MODE>(d, item, parity); break;
            case 6: batch_item<2, 4, MODE>(d, item, parity); break;
            case 7: batch_item<4, 1, MODE>(d, item, parity); break;
            case 8: batch_item<4, 2, MODE>(d, item, parity); break;
            default: batch_item<8, 1, MODE>(d, item, parity); break;
        }
    }
}

// Beliefs (Eq. 3) and MAP labels of every instance into concatenated outputs.
template <int LPL>
__device__ __forceinline__ void batch_readout_item(const InstDesc* __restrict__ d, const Item& item,
                                                   int parity, float* beliefs, int* labels) {
    constexpr int RPB = kBlock / kRow;
    const int lane = threadIdx.x & (kRow - 1);
    const int row = threadIdx.x / kRow;
    const int M = d->M;
    const size_t plane = (size_t)d->N * M;
    const bool full = M == kRow * LPL;
    const int x0 = lane * LPL;
    for (int pass = 0; pass < item.passes; ++pass) {
        const Pixel px = sync_pixel(item.first + pass * RPB + row, d->H, d->W, d->N);
        if (!px.ok) continue;
        PixelInputs<LPL> pin;
        load_pixel_ptr<LPL>(d->g, d->msg[parity], plane, M, px, x0, full, pin);
        float b[LPL];
        float z = 0.0f;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            b[i] = (((pin.g[i] * pin.m[kLeft][i]) * pin.m[kRight][i]) * pin.m[kUp][i]) * pin.m[kDown][i];
            z += b[i];
        }
        z = row_sum(z);
        const float inv = 1.0f / z;
        float best = -1.0f;
        int arg = 0x7fffffff;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            b[i] *= inv;
            if (x0 + i < M && b[i] > best) { best = b[i]; arg = x0 + i; }
        }
        if (beliefs) store_labels<LPL, false>(beliefs + d->belief_off + (size_t)px.p * M, x0, M, full, b);
        if (labels) {
#define BP_ARGMAX_STEP(CTRL)                                                   \
            {                                                                  \
                const float ob = dpp<CTRL>(best);                              \
                const int oa = dpp_i<CTRL>(arg);                               \
                if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; } \
            }
            BP_ARGMAX_STEP(kQuad1032)
            BP_ARGMAX_STEP(kQuad2301)
            BP_ARGMAX_STEP(kRowHalfMirror)
            BP_ARGMAX_STEP(kRowMirror)
#undef BP_ARGMAX_STEP
            if (lane == 0) labels[d->label_off + px.p] = arg;
        }
    }
}

__global__ __launch_bounds__(kBlock) void batch_readout_kernel(const InstDesc* __restrict__ inst,
                                                               const Item* __restrict__ items,
                                                               int n_items, int parity,
                                                               float* beliefs, int* labels) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = items[it];
        const InstDesc* d = inst + item.inst;
        const int arm = d->arm;  // arms 0-3: LPL 1, 4-6: LPL 2, 7-8: LPL 4, 9: LPL 8
        if (arm <= 3) batch_readout_item<1>(d, item, parity, beliefs, labels);
        else if (arm <= 6) batch_readout_item<2>(d, item, parity, beliefs, labels);
        else if (arm <= 8) batch_readout_item<4>(d, item, parity, beliefs, labels);
        else batch_readout_item<8>(d, item, parity, beliefs, labels);
    }
}

}  // namespace bpk
