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

// Code paths compiled into the batched kernel: (lanes per pixel G, window
// half-width TW); an instance with truncation T runs the smallest TW >= T
// for its G.  Every M <= 256 and T <= 8 has a path.
constexpr int kBatchClasses = 5;   // G = 4, 8, 16, 32, 64
constexpr int kBatchArms = 15;
constexpr int kArmG[kBatchArms] = {4, 4, 4, 8, 8, 8, 16, 16, 16, 32, 32, 32, 64, 64, 64};
constexpr int kArmTw[kBatchArms] = {2, 4, 8, 2, 4, 8, 2, 4, 8, 2, 4, 8, 2, 4, 8};

struct InstDesc {
    const float* g;          // unary [H][W][M]
    float* msg[2];           // ping-pong inbox planes [4][H][W][M]
    long long belief_off;    // offset of this instance in a concatenated beliefs array
    long long label_off;     // offset in a concatenated labels array
    int H, W, M, N, T;
    int arm;                 // index into kArmG / kArmTw
    float fbar;              // float32 (max-product)
    float tab_f[kBatchTab];  // f(d), |d| <= T (max-product, float32)
    double fbar_d;           // double (sum-product)
    double tab_wd[kBatchTab];  // f(d) - fbar, |d| <= T (sum-product, double)
};

struct Item {
    int inst;
    int first;               // first pixel (row-major) of the item
    int passes;              // passes of kBlock/G pixels (one pixel per G lanes)
    int pad;
};

template <int G, int TW, int MODE>
__device__ __forceinline__ void batch_item(const InstDesc* __restrict__ d, const Item& item, int parity) {
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const float* in = d->msg[parity];
    float* out = d->msg[parity ^ 1];
    const int M = d->M, W = d->W;
    const size_t plane = (size_t)d->N * M;
    const bool full = M == G * kLpl;
    const int x0 = pos * kLpl;
    const float* tab = d->tab_f;
    const float fbar = d->fbar;
    for (int pass = 0; pass < item.passes; ++pass) {
        const Pixel px = sync_pixel(item.first + pass * RPB + grp, d->H, W, d->N);
        if (!px.ok) continue;  // whole groups only
        PixelInputs pin;
        load_pixel_ptr(d->g, in, plane, M, px, x0, full, pin);
        double h[4][kLpl];
        make_h_d(pin, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[kLpl];
            if constexpr (MODE == kSum) sum_message_d<G, TW>(h[o], d->tab_wd, d->fbar_d, pos, M, x0, full, u);
            else max_message_d<G, TW>(h[o], tab, fbar, pos, M, x0, full, u);
            store_message(out, plane, M, W, px, o, x0, full, u);
        }
    }
}

// One persistent kernel per lane class G (the work queue is partitioned by
// class), so each kernel's register budget is that of its own three window
// variants rather than the union over every class.
template <int MODE, int G>
__global__ __launch_bounds__(kBlock) void batch_update_kernel(const InstDesc* __restrict__ inst,
                                                              const Item* __restrict__ items,
                                                              int n_items, int parity) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = items[it];
        const InstDesc* d = inst + item.inst;
        switch (d->arm % 3) {  // arms 3c, 3c+1, 3c+2: TW = 2, 4, 8 for class c
            case 0: batch_item<G, 2, MODE>(d, item, parity); break;
            case 1: batch_item<G, 4, MODE>(d, item, parity); break;
            default: batch_item<G, 8, MODE>(d, item, parity); break;
        }
    }
}

// Beliefs (Eq. 3) and MAP labels of every instance into concatenated outputs.
template <int G>
__device__ __forceinline__ void batch_readout_item(const InstDesc* __restrict__ d, const Item& item,
                                                   int parity, float* beliefs, int* labels) {
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int M = d->M;
    const size_t plane = (size_t)d->N * M;
    const bool full = M == G * kLpl;
    const int x0 = pos * kLpl;
    for (int pass = 0; pass < item.passes; ++pass) {
        const Pixel px = sync_pixel(item.first + pass * RPB + grp, d->H, d->W, d->N);
        if (!px.ok) continue;
        PixelInputs pin;
        load_pixel_ptr(d->g, d->msg[parity], plane, M, px, x0, full, pin);
        readout_pixel<G>(pin, M, x0, full, beliefs ? beliefs + d->belief_off + (size_t)px.p * M : nullptr,
                         labels ? labels + d->label_off + px.p : nullptr);
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void batch_readout_kernel(const InstDesc* __restrict__ inst,
                                                               const Item* __restrict__ items,
                                                               int n_items, int parity,
                                                               float* beliefs, int* labels) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item item = items[it];
        batch_readout_item<G>(inst + item.inst, item, parity, beliefs, labels);
    }
}

}  // namespace bpk
