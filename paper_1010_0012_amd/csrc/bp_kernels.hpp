// Kernel templates of the grid BP library.  Instantiated and launched from
// the bp_launch_*.hip translation units; declared for the host side in
// bp_launch.hpp.
#pragma once

#include "bp_device.hpp"

namespace bpk {

// Window gather: win[(K-J)*LPL + i] <- label (l-J)*LPL + i (lane l-J) and
// win[(K+J)*LPL + i] <- label (l+J)*LPL + i (lane l+J), for J = 1..K.  The
// DPP control is an immediate, hence the compile-time recursion.
template <int LPL, int K, int J>
__device__ __forceinline__ void fill_window(const float (&h)[LPL], float (&win)[(2 * K + 1) * LPL]) {
    if constexpr (J >= 1) {
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            win[(K - J) * LPL + i] = dpp<row_shr(J)>(h[i]);
            win[(K + J) * LPL + i] = dpp<row_shl(J)>(h[i]);
        }
        fill_window<LPL, K, J - 1>(h, win);
    }
}

// ------------------------------------------------ sparse O(mM) update ----
// One message p -> q with the paper's trick.
//   sum (Eq. 7):  u(y) = fbar * S + sum_{|d| <= T} (f(d) - fbar) * h(y + d),
//                 S = sum_x h(x), computed once per message;
//   max (Eq. 11): u(y) = max(fbar * Hm, max_{|d| <= T} f(d) * h(y + d)),
//                 Hm = max_x h(x), computed once per message.
// The window lives in registers: this lane's LPL labels plus K neighbouring
// lanes' labels on each side, fetched with DPP row shifts.  Labels outside
// the row read 0, which is also the clip at the ends of the label range
// (Nbd(y) stops at 0 and M-1).  Taps with T < |d| <= K*LPL carry weight 0,
// so rounding K up changes no result.
// Symmetric banded window: u[i] = base + sum_{|d| <= K*LPL} tab[|d|] * v(y_i + d)
// (sum) or max(base, max tab[|d|] * v(y_i + d)) (max), v read from this lane
// and K lanes each side (0 outside the row).
template <int LPL, int K, int MODE>
__device__ __forceinline__ void window_apply(const float (&v)[LPL], const float* tab, float base,
                                             float (&u)[LPL]) {
    constexpr int TW = K * LPL;
    constexpr int NW = (2 * K + 1) * LPL;
    float win[NW];
#pragma unroll
    for (int i = 0; i < LPL; ++i) win[K * LPL + i] = v[i];
    fill_window<LPL, K, K>(v, win);
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        float acc = base;
#pragma unroll
        for (int d = -TW; d <= TW; ++d) {
            const float w = tab[d < 0 ? -d : d];
            const float x = win[K * LPL + i + d];
            if constexpr (MODE == kSum) acc = fmaf(w, x, acc);
            else acc = fmaxf(acc, w * x);
        }
        u[i] = acc;
    }
}

// Row-wide sum (or max) of an LPL-per-lane vector; same bits on every lane.
template <int LPL, int MODE>
__device__ __forceinline__ float row_total(const float (&v)[LPL]) {
    float s = v[0];
#pragma unroll
    for (int i = 1; i < LPL; ++i) s = (MODE == kSum) ? s + v[i] : fmaxf(s, v[i]);
    return row_reduce<MODE>(s);
}

template <int LPL, int K, int MODE>
__device__ __forceinline__ void sparse_message(const float (&h)[LPL], const UpdateArgs& a,
                                               float (&u)[LPL]) {
    const float s = row_total<LPL, MODE>(h);  // the once-per-message term
    window_apply<LPL, K, MODE>(h, a.tab, a.fbar * s, u);
}

// Grid-wide update, register window.  One 16-lane row per sending pixel;
// each row handles P pixels, loading all of them before computing so that
// P times the bytes are in flight per wave.  Within a wave the four rows take
// consecutive pixels for each j, so every load and store stays contiguous.
template <int LPL, int K, int MODE, int P>
__global__ __launch_bounds__(kBlock) void sparse_update_kernel(UpdateArgs a) {
    constexpr int RPB = kBlock / kRow;  // rows per block
    const int lane = threadIdx.x & (kRow - 1);
    const int base = blockIdx.x * RPB * P + threadIdx.x / kRow;
    const int x0 = lane * LPL;
    const bool full = a.M == kRow * LPL;
    Pixel px[P];
    PixelInputs<LPL> in[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        px[j] = map_slot(base + j * RPB, a);
        if (px[j].ok) {
            load_pixel<LPL>(a, px[j], x0, full, in[j]);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                in[j].g[i] = 1.0f;
                in[j].m[0][i] = in[j].m[1][i] = in[j].m[2][i] = in[j].m[3][i] = 1.0f;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        float h[4][LPL];
        make_h<LPL>(in[j], h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[LPL];
            sparse_message<LPL, K, MODE>(h[o], a, u);
            normalise_store<LPL>(a, px[j], o, x0, full, u);
        }
    }
}

// ------------------------------------- sparse update, runtime window ----
// Same arithmetic for windows too wide for registers ((2K+1)*LPL large):
// h is staged in LDS per pixel and the compatible states of each y are
// visited with runtime bounds [max(0, y-T), min(M-1, y+T)].
template <int LPL, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_update_wide_kernel(UpdateArgs a) {
    extern __shared__ float lds[];             // [16 pixels][16*LPL] + tab[kMaxTab]
    constexpr int CAP = kRow * LPL;
    float* tab = lds + (kBlock / kRow) * CAP;
    for (int i = threadIdx.x; i < kMaxTab; i += kBlock) tab[i] = a.tab[i];
    const int lane = threadIdx.x & (kRow - 1);
    const int grp = threadIdx.x / kRow;
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / kRow;
    Pixel px = map_slot(slot, a);
    const int x0 = lane * LPL;
    const bool full = a.M == CAP;
    PixelInputs<LPL> in;
    if (px.ok) {
        load_pixel<LPL>(a, px, x0, full, in);
    } else {
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            in.g[i] = 1.0f;
            in.m[0][i] = in.m[1][i] = in.m[2][i] = in.m[3][i] = 1.0f;
        }
    }
    float h[4][LPL];
    make_h<LPL>(in, h);
    float* hs = lds + grp * CAP;
    __syncthreads();
#pragma unroll 1
    for (int o = 0; o < 4; ++o) {
        float s = h[o][0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) s = (MODE == kSum) ? s + h[o][i] : fmaxf(s, h[o][i]);
        s = row_reduce<MODE>(s);
#pragma unroll
        for (int i = 0; i < LPL; ++i) hs[x0 + i] = h[o][i];
        __syncthreads();
        const float base = a.fbar * s;
        float u[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const int y = x0 + i;
            const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
            float acc = base;
            for (int x = lo; x <= hi; ++x) {
                const float w = tab[x > y ? x - y : y - x];
                if constexpr (MODE == kSum) acc = fmaf(w, hs[x], acc);
                else acc = fmaxf(acc, w * hs[x]);
            }
            u[i] = acc;
        }
        __syncthreads();
        normalise_store<LPL>(a, px, o, x0, full, u);
    }
}

// ------------------------------------------ dense O(M^2) comparison ----
// Eq. 2 / Eq. 9 as written: u(y) = sum (or max) over every sender label x of
// F[x][y] * h(x), with F the full M x M float32 table (f(|x-y|) inside the
// window, fbar outside) staged in LDS once per workgroup.  h, the
// normalisation and the store are the same device functions as the sparse
// kernels, so max-product results match them bit for bit.
// Workgroups loop over 16-pixel tiles to amortise the table.
template <int LPL, int MODE>
__global__ __launch_bounds__(kBlock) void dense_update_kernel(UpdateArgs a) {
    extern __shared__ float lds[];  // F[M][CAP] then h[16 pixels][CAP][4]
    constexpr int CAP = kRow * LPL;
    float* F = lds;
    float* hs = lds + a.M * CAP;
    for (int i = threadIdx.x; i < a.M * CAP; i += kBlock) {
        const int x = i / CAP, y = i - x * CAP;
        const int d = x > y ? x - y : y - x;
        F[i] = (y >= a.M) ? 0.0f : (d <= a.T ? a.tab[d] : a.fbar);
    }
    const int lane = threadIdx.x & (kRow - 1);
    const int grp = threadIdx.x / kRow;
    const int x0 = lane * LPL;
    const bool full = a.M == CAP;
    const int n_tiles = (a.n_slots + kBlock / kRow - 1) / (kBlock / kRow);
    float* hg = hs + grp * CAP * 4;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int slot = tile * (kBlock / kRow) + grp;
        Pixel px = map_slot(slot, a);
        PixelInputs<LPL> in;
        if (px.ok) {
            load_pixel<LPL>(a, px, x0, full, in);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                in.g[i] = 1.0f;
                in.m[0][i] = in.m[1][i] = in.m[2][i] = in.m[3][i] = 1.0f;
            }
        }
        float h[4][LPL];
        make_h<LPL>(in, h);
        __syncthreads();  // previous tile done with hs (and F built on entry)
#pragma unroll
        for (int i = 0; i < LPL; ++i)
            *reinterpret_cast<float4*>(hg + (x0 + i) * 4) =
                make_float4(h[0][i], h[1][i], h[2][i], h[3][i]);
        __syncthreads();
        float u[4][LPL];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int i = 0; i < LPL; ++i) u[o][i] = 0.0f;
        for (int x = 0; x < a.M; ++x) {
            const float4 hv = *reinterpret_cast<const float4*>(hg + x * 4);
            const float* Fr = F + x * CAP + x0;
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const float f = Fr[i];
                if constexpr (MODE == kSum) {
                    u[0][i] = fmaf(f, hv.x, u[0][i]);
                    u[1][i] = fmaf(f, hv.y, u[1][i]);
                    u[2][i] = fmaf(f, hv.z, u[2][i]);
                    u[3][i] = fmaf(f, hv.w, u[3][i]);
                } else {
                    u[0][i] = fmaxf(u[0][i], f * hv.x);
                    u[1][i] = fmaxf(u[1][i], f * hv.y);
                    u[2][i] = fmaxf(u[2][i], f * hv.z);
                    u[3][i] = fmaxf(u[3][i], f * hv.w);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) normalise_store<LPL>(a, px, o, x0, full, u[o]);
    }
}

// ------------------------------------------------------------ readout ----
// Eq. 3: b = g * product of all incoming messages, normalised; MAP label =
// argmax of the normalised float32 beliefs, lowest label on ties.
template <int LPL>
__global__ __launch_bounds__(kBlock) void readout_kernel(UpdateArgs a, float* beliefs, int* labels) {
    const int lane = threadIdx.x & (kRow - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / kRow;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;
    const int x0 = lane * LPL;
    const bool full = a.M == kRow * LPL;
    PixelInputs<LPL> in;
    load_pixel<LPL>(a, px, x0, full, in);
    float b[LPL];
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        b[i] = (((in.g[i] * in.m[kLeft][i]) * in.m[kRight][i]) * in.m[kUp][i]) * in.m[kDown][i];
        z += b[i];
    }
    z = row_sum(z);
    const float inv = 1.0f / z;
    float best = -1.0f;
    int arg = 0x7fffffff;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        b[i] *= inv;
        if (x0 + i < a.M && b[i] > best) { best = b[i]; arg = x0 + i; }
    }
    if (beliefs) store_labels<LPL, false>(beliefs + (size_t)px.p * a.M, x0, a.M, full, b);
    if (labels) {
        // (value, index) tournament across the row: larger value wins, the
        // lower index breaks ties; the result is the same on every lane.
#define BP_ARGMAX_STEP(CTRL)                                               \
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
        if (lane == 0) labels[px.p] = arg;
    }
}

}  // namespace bpk
