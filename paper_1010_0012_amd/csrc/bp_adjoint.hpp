// Adjoint (reverse-mode derivative) of unrolled synchronous sum-product BP.
//
// Sum-product beliefs are smooth functions of the unary and of the potential,
// which is what marginal-based parameter learning needs (the paper motivates
// sum-product BP by maximum-likelihood / CRF estimation, Sec. 1 and Sec. 7).
// For a message e = p -> q with h from Eq. 5, u = F-product of h (Eq. 2,
// evaluated with the Eq. 7 split), Z = sum u and m = u / Z, and with
// lambda_e = dL/dlog m_e, one reverse step computes
//   mu   = lambda_e - m * sum(lambda_e)
//   ubar = mu / u                                  (dL/du)
//   hbar = fbar * sum(ubar) + sum_{|d|<=T} w(d) ubar(x+d)
//          (F applied from the other side; F is symmetric, so this is the
//           same banded window as the forward update, on ubar)
//   eta  = hbar * h                                (dL/dlog h)
//   theta_bar_p += sum over p's outgoing messages of eta
//   lambda^t_{k->p} = sum of eta over p's outgoing messages except to k
//   alpha_bar += fbar' * S * sum(ubar) + sum_y ubar(y) * sum_{|d|<=T} (f'(d) - fbar') h(y+d)
// with f'(d) = -|d| f(d) and fbar' = -T fbar when fbar is tied to f(T).
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

constexpr int kAdjTab = 32;  // taps the adjoint tables hold (|d| < 32)

struct AdjointArgs {
    const float* g;         // unary [N][M]
    const float* m;         // state m^t, inbox planes [4][N][M]
    const float* lam_in;    // dL/dlog m^{t+1}, inbox layout
    float* lam_out;         // dL/dlog m^t, inbox layout (null at t = 0)
    float* theta_bar;       // dL/dlog g [N][M], accumulated in place
    float* alpha_part;      // one partial per workgroup, accumulated in place
    int H, W, M, N;
    float fbar;
    float dfbar;            // d fbar / d alpha
    float w[kAdjTab];       // f(d) - fbar for |d| <= T, 0 beyond
    float dw[kAdjTab];      // f'(d) - fbar' for |d| <= T, 0 beyond
};

struct SeedArgs {
    const float* g;
    const float* m;         // final state m^n
    const float* dL_db;     // gradient of the loss w.r.t. the normalised beliefs [N][M]
    float* theta_bar;       // written: the direct term
    float* lam_out;         // written: lambda^n, inbox layout
    int H, W, M, N;
};

template <int LPL>
__device__ __forceinline__ void load_pixel_at(const float* g, const float* m, int N, int M,
                                              const Pixel& px, int x0, bool full,
                                              PixelInputs<LPL>& in) {
    if (!px.ok) {
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            in.g[i] = 1.0f;
            in.m[0][i] = in.m[1][i] = in.m[2][i] = in.m[3][i] = 1.0f;
        }
        return;
    }
    const size_t plane = (size_t)N * M;
    const size_t off = (size_t)px.p * M;
    load_labels<LPL, true>(g + off, x0, M, full, in.g, 0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (px.has[k]) {
            load_labels<LPL, true>(m + k * plane + off, x0, M, full, in.m[k], 1.0f);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) in.m[k][i] = 1.0f;
        }
    }
}

// lambda^n and the direct theta term from the loss gradient on the beliefs:
// with b = softmax of the log-belief, dL/dlogit = b * (dL/db - sum b dL/db).
template <int LPL>
__global__ __launch_bounds__(kBlock) void adjoint_seed_kernel(SeedArgs a) {
    const int lane = threadIdx.x & (kRow - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / kRow;
    const Pixel px = sync_pixel(slot, a.H, a.W, a.N);
    if (!px.ok) return;
    const int x0 = lane * LPL;
    const bool full = a.M == kRow * LPL;
    PixelInputs<LPL> in;
    load_pixel_at<LPL>(a.g, a.m, a.N, a.M, px, x0, full, in);
    float b[LPL], gb[LPL];
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        // same product order and normalisation as the readout kernel
        b[i] = (((in.g[i] * in.m[kLeft][i]) * in.m[kRight][i]) * in.m[kUp][i]) * in.m[kDown][i];
        z += b[i];
    }
    z = row_sum(z);
    const float inv = 1.0f / z;
    load_labels<LPL, false>(a.dL_db + (size_t)px.p * a.M, x0, a.M, full, gb, 0.0f);
    float dot = 0.0f;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        b[i] *= inv;
        dot = fmaf(b[i], gb[i], dot);
    }
    dot = row_sum(dot);
    float abar[LPL];
#pragma unroll
    for (int i = 0; i < LPL; ++i) abar[i] = b[i] * (gb[i] - dot);
    store_labels<LPL, false>(a.theta_bar + (size_t)px.p * a.M, x0, a.M, full, abar);
    const size_t plane = (size_t)a.N * a.M;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (px.has[k])
            store_labels<LPL, true>(a.lam_out + k * plane + (size_t)px.p * a.M, x0, a.M, full, abar);
}

// One reverse synchronous step (see the header comment).
template <int LPL, int K>
__global__ __launch_bounds__(kBlock) void adjoint_step_kernel(AdjointArgs a) {
    constexpr int RPB = kBlock / kRow;
    __shared__ float red[RPB];
    const int lane = threadIdx.x & (kRow - 1);
    const int row = threadIdx.x / kRow;
    const int slot = blockIdx.x * RPB + row;
    const Pixel px = sync_pixel(slot, a.H, a.W, a.N);
    const int x0 = lane * LPL;
    const bool full = a.M == kRow * LPL;
    const size_t plane = (size_t)a.N * a.M;
    PixelInputs<LPL> in;
    load_pixel_at<LPL>(a.g, a.m, a.N, a.M, px, x0, full, in);
    float h[4][LPL];
    make_h<LPL>(in, h);
    float eta[4][LPL];
    float alpha_pix = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const bool live = px.ok && px.has[o];
        float lam[LPL];
        if (live) {
            const int q = neighbour(px, o, a.W);
            load_labels<LPL, true>(a.lam_in + opposite(o) * plane + (size_t)q * a.M, x0, a.M, full, lam, 0.0f);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) lam[i] = 0.0f;
        }
        // forward recompute: u (Eq. 7), Z, m
        const float S = row_total<LPL, kSum>(h[o]);
        float u[LPL];
        window_apply<LPL, K, kSum>(h[o], a.w, a.fbar * S, u);
#pragma unroll
        for (int i = 0; i < LPL; ++i)
            if (!full && x0 + i >= a.M) u[i] = 0.0f;
        const float inv = 1.0f / row_total<LPL, kSum>(u);
        const float sl = row_total<LPL, kSum>(lam);
        float ub[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float mu = lam[i] - (u[i] * inv) * sl;
            ub[i] = (full || x0 + i < a.M) ? mu / u[i] : 0.0f;
        }
        const float su = row_total<LPL, kSum>(ub);
        float hb[LPL];
        window_apply<LPL, K, kSum>(ub, a.w, a.fbar * su, hb);
#pragma unroll
        for (int i = 0; i < LPL; ++i) eta[o][i] = hb[i] * h[o][i];
        float v[LPL];
        window_apply<LPL, K, kSum>(h[o], a.dw, 0.0f, v);
        float dot = 0.0f;
#pragma unroll
        for (int i = 0; i < LPL; ++i) dot = fmaf(ub[i], v[i], dot);
        dot = row_sum(dot);
        alpha_pix += fmaf(a.dfbar * S, su, dot);
    }
    if (px.ok) {
        float tb[LPL];
        float* tp = a.theta_bar + (size_t)px.p * a.M;
        load_labels<LPL, false>(tp, x0, a.M, full, tb, 0.0f);
#pragma unroll
        for (int i = 0; i < LPL; ++i)
            tb[i] += (eta[kLeft][i] + eta[kRight][i]) + (eta[kUp][i] + eta[kDown][i]);
        store_labels<LPL, false>(tp, x0, a.M, full, tb);
        if (a.lam_out) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!px.has[k]) continue;
                float lo[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    // every outgoing message of p except the one to k
                    const float lr = k < 2 ? eta[k ^ 1][i] : eta[kLeft][i] + eta[kRight][i];
                    const float ud = k < 2 ? eta[kUp][i] + eta[kDown][i] : eta[k ^ 1][i];
                    lo[i] = lr + ud;
                }
                store_labels<LPL, true>(a.lam_out + k * plane + (size_t)px.p * a.M, x0, a.M, full, lo);
            }
        }
    }
    if (lane == 0) red[row] = px.ok ? alpha_pix : 0.0f;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
#pragma unroll
        for (int r = 0; r < RPB; ++r) s += red[r];
        a.alpha_part[blockIdx.x] += s;
    }
}

}  // namespace bpk
