// Kernel templates of the grid BP library.  Instantiated and launched from
// the bp_launch_*.hip translation units; declared for the host side in
// bp_launch.hpp.
#pragma once

#include "bp_device.hpp"

namespace bpk {

// Window gather for a pixel group of G lanes: win[(K-J)*4 + i] <- label
// (pos-J)*4 + i and win[(K+J)*4 + i] <- label (pos+J)*4 + i, J = 1..K, 0 for
// lanes outside the group.  The DPP control is an immediate, hence the
// compile-time recursion; wide groups chain one-lane shifts.
template <int G, int K, int J>
__device__ __forceinline__ void fill_window(const float (&h)[kLpl], float (&win)[(2 * K + 1) * kLpl],
                                            int pos, float (&lo)[kLpl], float (&hi)[kLpl]) {
    if constexpr (J <= K) {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            if constexpr (G <= 16) {
                lo[i] = from_lower<G, J>(h[i], pos);
                hi[i] = from_upper<G, J>(h[i], pos);
            } else {
                lo[i] = lower1<G>(lo[i], pos);
                hi[i] = upper1<G>(hi[i], pos);
            }
            win[(K - J) * kLpl + i] = lo[i];
            win[(K + J) * kLpl + i] = hi[i];
        }
        fill_window<G, K, J + 1>(h, win, pos, lo, hi);
    }
}

// ------------------------------------------------ sparse O(mM) update ----
// One message p -> q with the paper's trick.
//   sum (Eq. 7):  u(y) = fbar * S + sum_{|d| <= T} (f(d) - fbar) * h(y + d),
//                 S = sum_x h(x), computed once per message;
//   max (Eq. 11): u(y) = max(fbar * Hm, max_{|d| <= T} f(d) * h(y + d)),
//                 Hm = max_x h(x), computed once per message.
// The window lives in registers: this lane's 4 labels plus the labels of
// K = ceil(TW / 4) neighbouring lanes on each side (gathers that no tap uses
// are dead code).  Labels outside the group read 0, which is also the clip
// at the ends of the label range (Nbd(y) stops at 0 and M-1).  A variant
// compiled for TW >= T runs the taps T < |d| <= TW with weight 0, so
// rounding TW up changes no result.
template <int TW>
constexpr int window_k() { return (TW + kLpl - 1) / kLpl; }

// Symmetric banded window: u[i] = base + sum_{|d| <= TW} tab[|d|] * v(y_i + d)
// (sum) or max(base, max tab[|d|] * v(y_i + d)) (max).
template <int G, int TW, int MODE>
__device__ __forceinline__ void window_apply(const float (&v)[kLpl], const float* tab, float base,
                                             int pos, float (&u)[kLpl]) {
    constexpr int K = window_k<TW>();
    static_assert(K < G, "window wider than the pixel group");
    constexpr int NW = (2 * K + 1) * kLpl;
    float win[NW];
    float lo[kLpl], hi[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        win[K * kLpl + i] = v[i];
        lo[i] = hi[i] = v[i];
    }
    fill_window<G, K, 1>(v, win, pos, lo, hi);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        float acc = base;
#pragma unroll
        for (int d = -TW; d <= TW; ++d) {
            const float w = tab[d < 0 ? -d : d];
            const float x = win[K * kLpl + i + d];
            if constexpr (MODE == kSum) acc = fmaf(w, x, acc);
            else acc = fmaxf(acc, w * x);
        }
        u[i] = acc;
    }
}

// Sum-product window in double: u[i] = base + sum_{|d| <= TW} dtab[|d|] *
// v(y_i + d), with the double weights and float32 h converted exactly to
// double, so the only roundings are the double FMAs.  On ill-conditioned
// loopy grids float32 weights or a float32 accumulation both showed belief
// errors near 1e-5 after 30 iterations; double weights and accumulation
// stay near 1e-6.
template <int G, int TW>
__device__ __forceinline__ void window_sum_d(const float (&v)[kLpl], const double* dtab, double base,
                                             int pos, double (&u)[kLpl]) {
    constexpr int K = window_k<TW>();
    static_assert(K < G, "window wider than the pixel group");
    constexpr int NW = (2 * K + 1) * kLpl;
    float win[NW];
    float lo[kLpl], hi[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        win[K * kLpl + i] = v[i];
        lo[i] = hi[i] = v[i];
    }
    fill_window<G, K, 1>(v, win, pos, lo, hi);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        double acc = base;
#pragma unroll
        for (int d = -TW; d <= TW; ++d) acc = fma(dtab[d < 0 ? -d : d], (double)win[K * kLpl + i + d], acc);
        u[i] = acc;
    }
}

// One sum-product message (Eq. 7) in double: S = sum h once per message,
// the window, Z and the normalisation in double, m rounded once to float.
template <int G, int TW>
__device__ __forceinline__ void sum_message_d(const float (&h)[kLpl], const double* dtab, double fbar, int pos,
                                              int M, int x0, bool full, float (&m)[kLpl]) {
    double s = ((double)h[0] + (double)h[1]) + ((double)h[2] + (double)h[3]);
    s = group_sum_d<G>(s);
    double u[kLpl];
    window_sum_d<G, TW>(h, dtab, fbar * s, pos, u);
    normalise_d<G>(u, M, x0, full, m);
}

// Double weights w(d) = f(d) - fbar for d <= T (f(d) = exp(-alpha d)) built
// on the device, for kernels whose windows reach past the argument table.
__device__ __forceinline__ double weight_d(const UpdateArgs& a, int d) {
    return d <= a.T ? exp(-a.alpha_d * d) - a.fbar_d : 0.0;
}

// Group-wide sum (or max) of a 4-per-lane vector; same bits on every lane.
template <int G, int MODE>
__device__ __forceinline__ float group_total(const float (&v)[kLpl]) {
    float s = v[0];
#pragma unroll
    for (int i = 1; i < kLpl; ++i) s = (MODE == kSum) ? s + v[i] : fmaxf(s, v[i]);
    return group_reduce<MODE, G>(s);
}

template <int G, int TW, int MODE>
__device__ __forceinline__ void sparse_message(const float (&h)[kLpl], const float* tab, float fbar,
                                               int pos, float (&u)[kLpl]) {
    const float s = group_total<G, MODE>(h);  // the once-per-message term
    window_apply<G, TW, MODE>(h, tab, fbar * s, pos, u);
}

// Grid-wide update, register window.  One group of G lanes per sending
// pixel; a wave's load and store instructions cover 64/G consecutive pixels.
template <int G, int TW, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_update_kernel(UpdateArgs a) {
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;  // whole groups only: no shuffle reads a retired lane's value
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    PixelInputs in;
    load_pixel(a, px, x0, full, in);
    float h[4][kLpl];
    make_h(in, h);
    const size_t plane = (size_t)a.N * a.M;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        float u[kLpl];
        if constexpr (MODE == kSum) {
            sum_message_d<G, TW>(h[o], a.dtab, a.fbar_d, pos, a.M, x0, full, u);
            store_message(a.out, plane, a.M, a.W, px, o, x0, full, u);
        } else {
            sparse_message<G, TW, MODE>(h[o], a.tab, a.fbar, pos, u);
            normalise_store<G>(a, px, o, x0, full, u);
        }
    }
}

// ------------------------------------- sparse update, runtime window ----
// Same arithmetic for windows wider than the compiled register variants:
// h is staged in LDS per pixel and the compatible states of each y are
// visited with runtime bounds [max(0, y-T), min(M-1, y+T)].
constexpr size_t wide_lds_bytes(int G) {
    return kMaxTab * sizeof(double) + kMaxTab * sizeof(float) + (size_t)(kBlock / G) * G * kLpl * sizeof(float);
}

template <int G, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_update_wide_kernel(UpdateArgs a) {
    extern __shared__ double lds_d[];  // dtab[kMaxTab] (sum), tab[kMaxTab] (max), h[kBlock/G][4G]
    constexpr int CAP = G * kLpl;
    double* dtab = lds_d;
    float* tab = reinterpret_cast<float*>(lds_d + kMaxTab);
    float* lds = tab + kMaxTab;
    for (int i = threadIdx.x; i < kMaxTab; i += kBlock) {
        if constexpr (MODE == kSum) dtab[i] = weight_d(a, i);
        else tab[i] = a.tab[i];
    }
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    PixelInputs in;
    if (px.ok) load_pixel(a, px, x0, full, in); else dummy_pixel(in);
    float h[4][kLpl];
    make_h(in, h);
    float* hs = lds + grp * CAP;
    __syncthreads();
#pragma unroll 1
    for (int o = 0; o < 4; ++o) {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) hs[x0 + i] = h[o][i];
        __syncthreads();
        float u[kLpl];
        if constexpr (MODE == kSum) {
            // double accumulation, as in the register variants
            double s = ((double)h[o][0] + (double)h[o][1]) + ((double)h[o][2] + (double)h[o][3]);
            s = group_sum_d<G>(s);
            const double base = a.fbar_d * s;
            double ud[kLpl];
#pragma unroll
            for (int i = 0; i < kLpl; ++i) {
                const int y = x0 + i;
                const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
                double acc = base;
                for (int x = lo; x <= hi; ++x) acc = fma(dtab[x > y ? x - y : y - x], (double)hs[x], acc);
                ud[i] = acc;
            }
            normalise_d<G>(ud, a.M, x0, full, u);
            __syncthreads();
            store_message(a.out, (size_t)a.N * a.M, a.M, a.W, px, o, x0, full, u);
        } else {
            const float base = a.fbar * group_total<G, MODE>(h[o]);
#pragma unroll
            for (int i = 0; i < kLpl; ++i) {
                const int y = x0 + i;
                const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
                float acc = base;
                for (int x = lo; x <= hi; ++x) acc = fmaxf(acc, tab[x > y ? x - y : y - x] * hs[x]);
                u[i] = acc;
            }
            __syncthreads();
            normalise_store<G>(a, px, o, x0, full, u);
        }
    }
}

// ------------------------------------------ dense O(M^2) comparison ----
// Eq. 2 / Eq. 9 as written: u(y) = sum (or max) over every sender label x of
// F[x][y] * h(x), with F the full M x M float32 table (f(|x-y|) inside the
// window, fbar outside) staged in LDS once per workgroup.  h, the
// normalisation and the store are the same device functions as the sparse
// kernels, so max-product results match them bit for bit.
// Workgroups loop over tiles of kBlock/G pixels to amortise the table.
// LDS of the dense kernel: sum-product keeps F in double (with a double
// f(d) table to build it from), max-product in float32; then h staging.
constexpr size_t dense_lds_bytes(int G, int M, int mode) {
    return mode == kSum
        ? kMaxTab * sizeof(double) + (size_t)M * G * kLpl * sizeof(double) + (size_t)kBlock * kLpl * 4 * sizeof(float)
        : (size_t)M * G * kLpl * sizeof(float) + (size_t)kBlock * kLpl * 4 * sizeof(float);
}

template <int G, int MODE>
__global__ __launch_bounds__(kBlock) void dense_update_kernel(UpdateArgs a) {
    extern __shared__ double lds_d[];
    constexpr int CAP = G * kLpl;
    constexpr int RPB = kBlock / G;
    double* Fd = lds_d + kMaxTab;                              // sum: F[M][4G] in double
    float* F = reinterpret_cast<float*>(lds_d);                // max: F[M][4G] in float32
    float* hs = MODE == kSum ? reinterpret_cast<float*>(Fd + a.M * CAP) : F + a.M * CAP;
    if constexpr (MODE == kSum) {
        double* fd = lds_d;                                    // f(d) = exp(-alpha d), d <= T
        for (int d = threadIdx.x; d < kMaxTab; d += kBlock) fd[d] = d <= a.T ? exp(-a.alpha_d * d) : 0.0;
        __syncthreads();
        for (int i = threadIdx.x; i < a.M * CAP; i += kBlock) {
            const int x = i / CAP, y = i - x * CAP;
            const int d = x > y ? x - y : y - x;
            Fd[i] = (y >= a.M) ? 0.0 : (d <= a.T ? fd[d] : a.fbar_d);
        }
    } else {
        for (int i = threadIdx.x; i < a.M * CAP; i += kBlock) {
            const int x = i / CAP, y = i - x * CAP;
            const int d = x > y ? x - y : y - x;
            F[i] = (y >= a.M) ? 0.0f : (d <= a.T ? a.tab[d] : a.fbar);
        }
    }
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    const int n_tiles = (a.n_slots + RPB - 1) / RPB;
    float* hg = hs + grp * CAP * 4;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const Pixel px = map_slot(tile * RPB + grp, a);
        PixelInputs in;
        if (px.ok) load_pixel(a, px, x0, full, in); else dummy_pixel(in);
        float h[4][kLpl];
        make_h(in, h);
        __syncthreads();  // previous tile done with hs (and F built on entry)
#pragma unroll
        for (int i = 0; i < kLpl; ++i)
            *reinterpret_cast<float4*>(hg + (x0 + i) * 4) = make_float4(h[0][i], h[1][i], h[2][i], h[3][i]);
        __syncthreads();
        if constexpr (MODE == kSum) {
            // same precision as the sparse sum-product update: double accumulation
            double u[4][kLpl];
#pragma unroll
            for (int o = 0; o < 4; ++o)
#pragma unroll
                for (int i = 0; i < kLpl; ++i) u[o][i] = 0.0;
            for (int x = 0; x < a.M; ++x) {
                const float4 hv = *reinterpret_cast<const float4*>(hg + x * 4);
                const double2 f01 = *reinterpret_cast<const double2*>(Fd + x * CAP + x0);
                const double2 f23 = *reinterpret_cast<const double2*>(Fd + x * CAP + x0 + 2);
                const double hd[4] = {(double)hv.x, (double)hv.y, (double)hv.z, (double)hv.w};
                const double fd[kLpl] = {f01.x, f01.y, f23.x, f23.y};
#pragma unroll
                for (int i = 0; i < kLpl; ++i)
#pragma unroll
                    for (int o = 0; o < 4; ++o) u[o][i] = fma(fd[i], hd[o], u[o][i]);
            }
            const size_t plane = (size_t)a.N * a.M;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float m[kLpl];
                normalise_d<G>(u[o], a.M, x0, full, m);
                store_message(a.out, plane, a.M, a.W, px, o, x0, full, m);
            }
        } else {
            float u[4][kLpl];
#pragma unroll
            for (int o = 0; o < 4; ++o)
#pragma unroll
                for (int i = 0; i < kLpl; ++i) u[o][i] = 0.0f;
            for (int x = 0; x < a.M; ++x) {
                const float4 hv = *reinterpret_cast<const float4*>(hg + x * 4);
                const float4 fr = *reinterpret_cast<const float4*>(F + x * CAP + x0);
                const float f4[kLpl] = {fr.x, fr.y, fr.z, fr.w};
#pragma unroll
                for (int i = 0; i < kLpl; ++i) {
                    const float f = f4[i];
                    u[0][i] = fmaxf(u[0][i], f * hv.x);
                    u[1][i] = fmaxf(u[1][i], f * hv.y);
                    u[2][i] = fmaxf(u[2][i], f * hv.z);
                    u[3][i] = fmaxf(u[3][i], f * hv.w);
                }
            }
#pragma unroll
            for (int o = 0; o < 4; ++o) normalise_store<G>(a, px, o, x0, full, u[o]);
        }
    }
}

// ------------------------------------------------------------ readout ----
// Eq. 3: b = g * product of all incoming messages, normalised; MAP label =
// argmax of the normalised float32 beliefs, lowest label on ties.
template <int G>
__device__ __forceinline__ void readout_pixel(const PixelInputs& in, int M, int x0, bool full,
                                              float* beliefs_row, int* label) {
    float b[kLpl];
    make_belief(in, b);
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) z += b[i];
    z = group_sum<G>(z);
    const float inv = 1.0f / z;
    float best = -1.0f;
    int arg = 0x7fffffff;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        b[i] *= inv;
        if (x0 + i < M && b[i] > best) { best = b[i]; arg = x0 + i; }
    }
    if (beliefs_row) store_labels<false>(beliefs_row, x0, M, full, b);
    if (label) {
        group_argmax<G>(best, arg);
        if (x0 == 0) *label = arg;
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void readout_kernel(UpdateArgs a, float* beliefs, int* labels) {
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    PixelInputs in;
    load_pixel(a, px, x0, full, in);
    readout_pixel<G>(in, a.M, x0, full, beliefs ? beliefs + (size_t)px.p * a.M : nullptr,
                     labels ? labels + px.p : nullptr);
}

}  // namespace bpk
