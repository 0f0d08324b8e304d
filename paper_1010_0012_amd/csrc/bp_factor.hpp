// Factor-graph BP with sparse-compatible higher-order factors (Sec. 7): a
// factor of arity K (2 or 3) equals a constant fbar except on a set C of
// compatible tuples, and its message update costs O(C + M) instead of the
// O(M^K) of visiting every completion.
//   variable -> factor: n_{v->a} = g_v * product of v's other incoming factor
//                       messages (adjacency order), normalised;
//   factor -> variable: sum: fbar * prod_{j != i} S_j + sum over the tuples
//                       with x_i = x of (f - fbar) * prod_{j != i} n_j(t_j);
//                       max: max(fbar * prod_{j != i} H_j, max over those
//                       tuples of f * prod_{j != i} n_j(t_j)),
// with S_j = sum n_j and H_j = max n_j (the factor analogue of Eq. 7 and
// Eq. 11; the max form needs f >= fbar on C).  Products run left to right
// in double; every message is normalised in double and rounded once.
//
// Tables: per type and slot i, the tuples grouped by their label at slot i
// (CSR rows, tuple order kept within a row); each entry holds the labels of
// the other slots in slot order, f (float32) and f - fbar (double).  A
// complete list of every tuple with fbar = 0 turns the same kernel into the
// plain O(M^K) update.
#pragma once

#include "bp_kernels.hpp"

namespace bpk {

constexpr int kFgMaxTypes = 16;

struct FgArgs {
    const float* g;          // [n_vars][M]
    const int* var_ptr;      // [n_vars + 1]
    const int* var_adj;      // slots a * 3 + i incident to each variable, in factor order
    const int* fac_type;     // [n_factors]
    const int* tptr;         // [n_types][3][M + 1] CSR rows per type and slot
    const int2* ent_o;       // labels of the other slots (second is -1 for arity 2)
    const float* ent_f;      // f(tuple)
    const double* ent_w;     // f(tuple) - fbar
    float* m_fv;             // [n_factors * 3][M] factor -> variable
    float* n_vf;             // [n_factors * 3][M] variable -> factor
    int n_vars, n_factors, M;
    int arity[kFgMaxTypes];
    float fbar[kFgMaxTypes];
};

// variable -> factor: one group of G lanes per variable.
template <int G>
__global__ __launch_bounds__(kBlock) void fg_var_kernel(FgArgs a) {
    const int pos = threadIdx.x & (G - 1);
    const int v = (blockIdx.x * kBlock + threadIdx.x) / G;
    if (v >= a.n_vars) return;  // whole groups
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    float gv[kLpl];
    load_labels<false>(a.g + (size_t)v * a.M, x0, a.M, full, gv, 0.0f);
    const int b0 = a.var_ptr[v], b1 = a.var_ptr[v + 1];
    for (int s = b0; s < b1; ++s) {
        double p[kLpl];
#pragma unroll
        for (int i = 0; i < kLpl; ++i) p[i] = gv[i];
        for (int t = b0; t < b1; ++t) {
            if (t == s) continue;
            float mv[kLpl];
            load_labels<false>(a.m_fv + (size_t)a.var_adj[t] * a.M, x0, a.M, full, mv, 0.0f);
#pragma unroll
            for (int i = 0; i < kLpl; ++i) p[i] *= mv[i];
        }
        float n[kLpl];
        normalise_d<G>(p, a.M, x0, full, n);
        store_labels<false>(a.n_vf + (size_t)a.var_adj[s] * a.M, x0, a.M, full, n);
    }
}

constexpr size_t fg_lds_bytes(int G) { return (size_t)(kBlock / G) * 2 * G * kLpl * sizeof(double); }

// factor -> variable: one group per (factor, slot); the other slots' incoming
// messages are staged in LDS for the tuple gathers.
template <int G, int MODE>
__global__ __launch_bounds__(kBlock) void fg_factor_kernel(FgArgs a) {
    extern __shared__ double lds_d[];
    constexpr int CAP = G * kLpl;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int item = (blockIdx.x * kBlock + threadIdx.x) / G;  // a * 3 + i
    const int fa = item / 3, i = item - 3 * (item / 3);
    const bool live_f = fa < a.n_factors;
    const int k = live_f ? a.fac_type[fa] : 0;
    const int K = a.arity[k];
    const bool live = live_f && i < K;
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    double* nj[2] = {lds_d + (size_t)grp * 2 * CAP, lds_d + (size_t)grp * 2 * CAP + CAP};
    // the other slots in slot order
    const int j0 = i == 0 ? 1 : 0;
    const int j1 = i == 2 ? 1 : 2;
    const int n_oth = K - 1;
    double agg[2] = {1.0, 1.0};
    for (int q = 0; q < 2; ++q) {
        float v[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (live && q < n_oth) load_labels<false>(a.n_vf + ((size_t)fa * 3 + (q ? j1 : j0)) * a.M, x0, a.M, full, v, 0.0f);
#pragma unroll
        for (int l = 0; l < kLpl; ++l) nj[q][x0 + l] = v[l];
        double r = MODE == kSum ? ((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3])
                                : fmax(fmax((double)v[0], (double)v[1]), fmax((double)v[2], (double)v[3]));
        r = MODE == kSum ? group_sum_d<G>(r) : group_max_d<G>(r);
        agg[q] = r;
    }
    __syncthreads();
    if (!live) return;  // after the only barrier
    // fbar term, products left to right
    double base = (double)a.fbar[k] * agg[0];
    if (n_oth == 2) base *= agg[1];
    const int* row = a.tptr + ((size_t)k * 3 + i) * (a.M + 1);
    double u[kLpl];
#pragma unroll
    for (int l = 0; l < kLpl; ++l) {
        const int x = x0 + l;
        double acc = base;
        if (x < a.M) {
            for (int e = row[x]; e < row[x + 1]; ++e) {
                const int2 o = a.ent_o[e];
                double p = MODE == kSum ? a.ent_w[e] : (double)a.ent_f[e];
                p *= nj[0][o.x];
                if (n_oth == 2) p *= nj[1][o.y];
                acc = MODE == kSum ? acc + p : fmax(acc, p);
            }
        }
        u[l] = acc;
    }
    float m[kLpl];
    normalise_d<G>(u, a.M, x0, full, m);
    store_labels<false>(a.m_fv + (size_t)item * a.M, x0, a.M, full, m);
}

// Beliefs (g times every incoming factor message, normalised in double) and
// MAP labels (argmax of the float32 beliefs, lowest label on ties).
template <int G>
__global__ __launch_bounds__(kBlock) void fg_belief_kernel(FgArgs a, float* beliefs, int* labels) {
    const int pos = threadIdx.x & (G - 1);
    const int v = (blockIdx.x * kBlock + threadIdx.x) / G;
    if (v >= a.n_vars) return;
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    float gv[kLpl];
    load_labels<false>(a.g + (size_t)v * a.M, x0, a.M, full, gv, 0.0f);
    double p[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) p[i] = gv[i];
    for (int t = a.var_ptr[v]; t < a.var_ptr[v + 1]; ++t) {
        float mv[kLpl];
        load_labels<false>(a.m_fv + (size_t)a.var_adj[t] * a.M, x0, a.M, full, mv, 0.0f);
#pragma unroll
        for (int i = 0; i < kLpl; ++i) p[i] *= mv[i];
    }
    float b[kLpl];
    normalise_d<G>(p, a.M, x0, full, b);
    if (beliefs) store_labels<false>(beliefs + (size_t)v * a.M, x0, a.M, full, b);
    if (labels) {
        float best = -1.0f;
        int arg = 1 << 30;
#pragma unroll
        for (int i = 0; i < kLpl; ++i)
            if (x0 + i < a.M && b[i] > best) { best = b[i]; arg = x0 + i; }
        group_argmax<G>(best, arg);
        if (pos == 0) labels[v] = arg;
    }
}

}  // namespace bpk
