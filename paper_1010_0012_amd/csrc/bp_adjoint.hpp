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
    float w[kAdjTab];       // f(d) - fbar for |d| <= T, 0 beyond (float32, the transposed window)
    float dw[kAdjTab];      // f'(d) - fbar' for |d| <= T, 0 beyond
    double fbar_d;          // forward recompute in double, as in the forward update
    double wd[kAdjTab];     // f(d) - fbar in double
};

struct SeedArgs {
    const float* g;
    const float* m;         // final state m^n
    const float* dL_db;     // gradient of the loss w.r.t. the normalised beliefs [N][M]
    float* theta_bar;       // written: the direct term
    float* lam_out;         // written: lambda^n, inbox layout
    int H, W, M, N;
};

__device__ __forceinline__ void load_pixel_at(const float* g, const float* m, int N, int M,
                                              const Pixel& px, int x0, bool full, PixelInputs& in) {
    if (px.ok) load_pixel_ptr(g, m, (size_t)N * M, M, px, x0, full, in);
    else dummy_pixel(in);
}

// lambda^n and the direct theta term from the loss gradient on the beliefs:
// with b = softmax of the log-belief, dL/dlogit = b * (dL/db - sum b dL/db).
template <int G>
__global__ __launch_bounds__(kBlock) void adjoint_seed_kernel(SeedArgs a) {
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = sync_pixel(slot, a.H, a.W, a.N);
    if (!px.ok) return;
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    PixelInputs in;
    load_pixel_at(a.g, a.m, a.N, a.M, px, x0, full, in);
    float b[kLpl], gb[kLpl];
    belief_d<G>(in, a.M, x0, full, b);  // the beliefs the readout returns, bit for bit
    load_labels<false>(a.dL_db + (size_t)px.p * a.M, x0, a.M, full, gb, 0.0f);
    float dot = 0.0f;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) dot = fmaf(b[i], gb[i], dot);
    dot = group_sum<G>(dot);
    float abar[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) abar[i] = b[i] * (gb[i] - dot);
    store_labels<false>(a.theta_bar + (size_t)px.p * a.M, x0, a.M, full, abar);
    const size_t plane = (size_t)a.N * a.M;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (px.has[k]) store_labels<true>(a.lam_out + k * plane + (size_t)px.p * a.M, x0, a.M, full, abar);
}

// A read-only row of zeros: the adjoint of a message that does not exist.
struct ZeroRow {
    float v[kMaxTab];
};
static __device__ ZeroRow kZeroRow = ZeroRow();  // never written

// One reverse synchronous step (see the header comment).  FULL: M == 4G.
// Loads are unconditional: a missing inbox row is read from the row of ones
// and a missing neighbour's adjoint from the row of zeros, and a slot past
// the last pixel reads pixel 0 (and stores nothing), so that every load of
// the group sits in one basic block.
template <int G, int TW, bool FULL>
__global__ __launch_bounds__(kBlock) void adjoint_step_kernel(AdjointArgs a) {
    constexpr int RPB = kBlock / G;
    __shared__ float red[RPB];
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int slot = blockIdx.x * RPB + grp;
    const Pixel px = sync_pixel(slot, a.H, a.W, a.N);
    const int x0 = pos * kLpl;
    constexpr bool full = FULL;
    const size_t plane = (size_t)a.N * a.M;
    const size_t off = px.ok ? (size_t)px.p * a.M : 0;
    PixelInputs in;
    load_labels<kUnaryNT>(a.g + off, x0, a.M, FULL, in.g, 0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float* row = px.ok && px.has[k] ? a.m + k * plane + off : kOnesRow.v;
        load_labels<kMsgNT>(row, x0, a.M, FULL, in.m[k], 1.0f);
    }
    float h[4][kLpl];
    make_h(in, h);
    double hd[4][kLpl];  // the forward update's h, for the recompute of u
    make_h_d(in, hd);
    float eta[4][kLpl];
    float alpha_pix = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const bool live = px.ok && px.has[o];
        float lam[kLpl];
        {
            const float* row =
                live ? a.lam_in + opposite(o) * plane + (size_t)neighbour(px, o, a.W) * a.M : kZeroRow.v;
            load_labels<true>(row, x0, a.M, FULL, lam, 0.0f);
        }
        // forward recompute: u (Eq. 7), Z, m, accumulated in double as in the
        // forward update
        double sd = (hd[o][0] + hd[o][1]) + (hd[o][2] + hd[o][3]);
        sd = group_sum_d<G>(sd);
        double ud[kLpl];
        window_sum_d<G, TW>(hd[o], a.wd, a.fbar_d * sd, pos, ud);
        double zd = 0.0;
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            if (!full && x0 + i >= a.M) ud[i] = 0.0;
            zd += ud[i];
        }
        const double inv = recip_d(group_sum_d<G>(zd));  // the forward's normaliser, bit for bit
        const float S = (float)sd;
        const float sl = group_total<G, kSum>(lam);
        float ub[kLpl];
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            const float mu = lam[i] - (float)(ud[i] * inv) * sl;
            ub[i] = (full || x0 + i < a.M) ? (float)((double)mu * recip_d(ud[i])) : 0.0f;
        }
        const float su = group_total<G, kSum>(ub);
        float hb[kLpl];
        window_apply<G, TW, kSum>(ub, a.w, a.fbar * su, pos, hb);
#pragma unroll
        for (int i = 0; i < kLpl; ++i) eta[o][i] = hb[i] * h[o][i];
        float v[kLpl];
        window_apply<G, TW, kSum>(h[o], a.dw, 0.0f, pos, v);
        float dot = 0.0f;
#pragma unroll
        for (int i = 0; i < kLpl; ++i) dot = fmaf(ub[i], v[i], dot);
        dot = group_sum<G>(dot);
        alpha_pix += fmaf(a.dfbar * S, su, dot);
    }
    if (px.ok) {
        float tb[kLpl];
        float* tp = a.theta_bar + (size_t)px.p * a.M;
        load_labels<false>(tp, x0, a.M, FULL, tb, 0.0f);
#pragma unroll
        for (int i = 0; i < kLpl; ++i)
            tb[i] += (eta[kLeft][i] + eta[kRight][i]) + (eta[kUp][i] + eta[kDown][i]);
        store_labels<false>(tp, x0, a.M, FULL, tb);
        if (a.lam_out) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!px.has[k]) continue;
                float lo[kLpl];
#pragma unroll
                for (int i = 0; i < kLpl; ++i) {
                    // every outgoing message of p except the one to k
                    const float lr = k < 2 ? eta[k ^ 1][i] : eta[kLeft][i] + eta[kRight][i];
                    const float ud = k < 2 ? eta[kUp][i] + eta[kDown][i] : eta[k ^ 1][i];
                    lo[i] = lr + ud;
                }
                store_labels<true>(a.lam_out + k * plane + (size_t)px.p * a.M, x0, a.M, FULL, lo);
            }
        }
    }
    if (pos == 0) red[grp] = px.ok ? alpha_pix : 0.0f;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
#pragma unroll
        for (int r = 0; r < RPB; ++r) s += red[r];
        a.alpha_part[blockIdx.x] += s;
    }
}

}  // namespace bpk
