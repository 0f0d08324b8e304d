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
// Max-product with some f < fbar in C takes the split form (Eq. 10's
// analogue): fbar times the largest product over the completions outside
// C.  With the other slots j < k, that maximum is, over first labels a, the
// product with the largest n_k(b) such that (a, b) is not listed: for an a
// with no listed tuple it is max n_k, and the best such a is the first
// entry of n_j's top list outside the listed a's; for a listed a it is the
// first entry of n_k's top list outside that a's listed b's.  Products keep
// the dense form's order, (fbar n_j(a)) n_k(b), and rounding is monotone, so
// the result equals the dense O(M^K) max bit for bit.
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
constexpr int kFgTop = 32;  // longest top list of the split form

struct FgArgs {
    const float* g;          // [n_vars][M]
    const int* var_ptr;      // [n_vars + 1]
    const int* var_adj;      // slots a * 3 + i incident to each variable, in factor order
    const int* fac_type;     // [n_factors]
    const int* tptr;         // [n_types][3][M + 1] CSR rows per type and slot
    const int2* ent_o;       // labels of the other slots (second is -1 for arity 2)
    const float* ent_f;      // f(tuple)
    const double* ent_w;     // f(tuple) - fbar
    const int2* ent_s;       // the other slots' labels of each row sorted (a, b), for membership tests
    float* m_fv;             // [n_factors * 3][M] factor -> variable
    float* n_vf;             // [n_factors * 3][M] variable -> factor
    const int* items;        // factor messages a * 3 + i grouped by (type, slot), each run padded with -1
                             // to a multiple of kFgLane items, so a workgroup's messages share one table
    int n_items;
    int n_vars, n_factors, M;
    int arity[kFgMaxTypes];
    float fbar[kFgMaxTypes];
    int eq10[kFgMaxTypes];          // max-product takes the split form (some f < fbar in C)
    int top[kFgMaxTypes][3][2];     // per slot: top-list lengths for the first and second other slot
};

// variable -> factor: one group of G lanes per variable.  Up to kFgCache
// incoming messages are loaded once into registers (statically indexed);
// the products keep the adjacency order either way.
constexpr int kFgCache = 8;

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
    const int deg = b1 - b0;
    if (deg <= kFgCache) {
        float c[kFgCache][kLpl];
#pragma unroll
        for (int q = 0; q < kFgCache; ++q)
            if (q < deg) load_labels<false>(a.m_fv + (size_t)a.var_adj[b0 + q] * a.M, x0, a.M, full, c[q], 0.0f);
        for (int s = 0; s < deg; ++s) {
            double p[kLpl];
#pragma unroll
            for (int i = 0; i < kLpl; ++i) p[i] = gv[i];
#pragma unroll
            for (int q = 0; q < kFgCache; ++q)
                if (q < deg && q != s)
#pragma unroll
                    for (int i = 0; i < kLpl; ++i) p[i] *= c[q][i];
            float n[kLpl];
            normalise_d<G>(p, a.M, x0, full, n);
            store_labels<false>(a.n_vf + (size_t)a.var_adj[b0 + s] * a.M, x0, a.M, full, n);
        }
        return;
    }
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

// Per group: the other slots' messages (2 x 4G doubles), then the split
// form's two top lists (values, then labels); after them, when the
// workgroup stages its table, the values (double) and the other slots'
// labels of its (type, slot) rows.
constexpr size_t fg_lds_bytes(int G, bool split) {
    return (size_t)(kBlock / G) * (2 * G * kLpl * sizeof(double) +
                                   (split ? 2 * kFgTop * (sizeof(double) + sizeof(int)) : 0));
}
constexpr size_t kFgStageBytes = 64 * 1024;  // LDS per workgroup when the table is staged
constexpr size_t fg_stage_entries(int G, bool split) {
    return (kFgStageBytes - fg_lds_bytes(G, split)) / (sizeof(double) + sizeof(int2));
}

// Is label x among the first slot's labels (w = 0) or the second's (w = 1)
// of entries [e0, e1) of the sorted list?
__device__ __forceinline__ bool listed(const int2* s, int e0, int e1, int x, int w) {
    for (int e = e0; e < e1; ++e)
        if ((w ? s[e].y : s[e].x) == x) return true;
    return false;
}

// factor -> variable: one group per (factor, slot); the other slots' incoming
// messages are staged in LDS for the tuple gathers.
// The split form's second term for one label of slot i: fbar times the
// largest product over the completions outside the label's listed tuples
// [e0, e1) (ent_s, sorted by (a, b)), or 0 when every completion is listed.
// top_v / top_i: the other slots' top lists ([0]: first other slot, [kFgTop]:
// second), n0: the first other slot's message (row_slot layout).
template <int G>
__device__ __forceinline__ double split_outside(const FgArgs& a, int k, int i, int e0, int e1, int n_oth,
                                               const double* n0, const double* top_v, const int* top_i) {
    const double fb = (double)a.fbar[k];
    const int2* s = a.ent_s;
    double best = 0.0;
    // first labels a with no listed tuple: the best is the first of the first
    // other slot's list outside the listed a's, with the largest n_k
    for (int r = 0; r < a.top[k][i][0]; ++r) {
        if (!listed(s, e0, e1, top_i[r], 0)) {
            double p = fb * top_v[r];
            if (n_oth == 2) p *= top_v[kFgTop];
            best = fmax(best, p);
            break;
        }
    }
    if (n_oth == 2) {
        // each listed a: the first of the second slot's list outside its b's
        for (int e = e0; e < e1;) {
            const int x = s[e].x;
            int f = e;
            while (f < e1 && s[f].x == x) ++f;
            for (int r = 0; r < a.top[k][i][1]; ++r) {
                if (!listed(s, e, f, top_i[kFgTop + r], 1)) {
                    best = fmax(best, (fb * n0[row_slot<G>(x)]) * top_v[kFgTop + r]);
                    break;
                }
            }
            e = f;
        }
    }
    return best;
}

// STAGE: the workgroup first copies its (type, slot) table rows to LDS
// (values as double: f - fbar for sum, f for max; the other slots' labels as
// their positions in the nj rows), so the per-entry reads of every message
// are LDS reads, shared by all of its groups, with no index arithmetic.
template <int G, int MODE, bool EQ10, bool STAGE>
__global__ __launch_bounds__(kBlock) void fg_factor_kernel(FgArgs a) {
    extern __shared__ double lds_d[];
    constexpr int CAP = G * kLpl;
    constexpr int RPB = kBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int item = a.items[blockIdx.x * RPB + grp];  // a * 3 + i, or -1
    const bool live = item >= 0;
    const int fa = live ? item / 3 : 0, i = live ? item - 3 * (item / 3) : 0;
    const int k = live ? a.fac_type[fa] : 0;
    const int K = a.arity[k];
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    double* nj[2] = {lds_d + (size_t)grp * 2 * CAP, lds_d + (size_t)grp * 2 * CAP + CAP};
    constexpr bool kTops = EQ10 && MODE == kMax;
    double* top_v = lds_d + (size_t)RPB * 2 * CAP + (size_t)grp * 2 * kFgTop;  // [2][kFgTop]
    int* top_i = reinterpret_cast<int*>(lds_d + (size_t)RPB * 2 * CAP + (size_t)RPB * 2 * kFgTop) + grp * 2 * kFgTop;
    const bool split = kTops && a.eq10[k];
    // the workgroup's table: every run of items starts a workgroup with a real
    // item, and a workgroup of padding only (runs are padded to 64 items) exits
    const int first = a.items[blockIdx.x * RPB];
    if (first < 0) return;  // whole workgroup, before the barrier
    const int* row0 = a.tptr + ((size_t)a.fac_type[first / 3] * 3 + first % 3) * (a.M + 1);
    const int e_base = row0[0];
    double* st_w = lds_d + fg_lds_bytes(G, kTops) / sizeof(double);
    int2* st_o = reinterpret_cast<int2*>(st_w + (row0[a.M] - e_base));
    if constexpr (STAGE) {
        for (int e = threadIdx.x; e < row0[a.M] - e_base; e += kBlock) {
            st_w[e] = MODE == kSum ? a.ent_w[e_base + e] : (double)a.ent_f[e_base + e];
            const int2 o = a.ent_o[e_base + e];
            st_o[e] = make_int2(row_slot<G>(o.x), row_slot<G>(o.y));  // the labels' slots in the nj rows
        }
    }
    // the other slots in slot order
    const int j0 = i == 0 ? 1 : 0;
    const int j1 = i == 2 ? 1 : 2;
    const int n_oth = K - 1;
    double agg[2] = {1.0, 1.0};
    for (int q = 0; q < 2; ++q) {
        float v[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (live && q < n_oth) load_labels<false>(a.n_vf + ((size_t)fa * 3 + (q ? j1 : j0)) * a.M, x0, a.M, full, v, 0.0f);
#pragma unroll
        for (int l = 0; l < kLpl; ++l) nj[q][l * G + pos] = v[l];  // row_slot layout
        double r = MODE == kSum ? ((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3])
                                : fmax(fmax((double)v[0], (double)v[1]), fmax((double)v[2], (double)v[3]));
        r = MODE == kSum ? group_sum_d<G>(r) : group_max_d<G>(r);
        agg[q] = r;
        if (split && q < n_oth) {  // this slot's top list, value descending
            const double vd[kLpl] = {v[0], v[1], v[2], v[3]};
            group_top_k<G>(vd, a.M, x0, pos, a.top[k][i][q], top_v + q * kFgTop, top_i + q * kFgTop);
        }
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
        double acc = split ? 0.0 : base;  // the split form replaces the fbar * prod H term
        if (x < a.M) {
            for (int e = row[x]; e < row[x + 1]; ++e) {
                int2 o;
                if constexpr (STAGE) {
                    o = st_o[e - e_base];
                } else {
                    o = a.ent_o[e];
                    o = make_int2(row_slot<G>(o.x), row_slot<G>(o.y));
                }
                double p = STAGE ? st_w[e - e_base] : MODE == kSum ? a.ent_w[e] : (double)a.ent_f[e];
                p *= nj[0][o.x];
                if (n_oth == 2) p *= nj[1][o.y];
                acc = MODE == kSum ? acc + p : fmax(acc, p);
            }
            if (split) acc = fmax(acc, split_outside<G>(a, k, i, row[x], row[x + 1], n_oth, nj[0], top_v, top_i));
        }
        u[l] = acc;
    }
    float m[kLpl];
    normalise_d<G>(u, a.M, x0, full, m);
    store_labels<false>(a.m_fv + (size_t)item * a.M, x0, a.M, full, m);
}

// factor -> variable with one message per lane, for M <= MM (16 or 32) and
// the sum and plain max forms: a workgroup is one wave of kFgLane items of
// one (type, slot) (runs are padded to whole workgroups), so the table entry
// of every step is the same for all lanes: uniform (scalar) reads of its
// labels and value, from the scalar cache or L2.  (Staging the table in LDS
// for workgroups of four waves sharing it measured no faster, 273 against
// 269 us per iteration at 256 x 256, M = 32; one packed 16-byte read per
// entry was slower, 290 us.)  Each lane gathers from its own copy of the
// other slots' messages, held in registers and indexed by the wave-uniform
// label.  The arithmetic is fg_factor_kernel's in the same order: S_j (H_j)
// as the group's tree over 4-label partials, the listed tuples of each label
// in row order with left-to-right products, and the normaliser as the same
// tree over the lanes of a G-lane group (G = lanes_for(M)), so the messages
// are the same bits.
constexpr int kFgLane = 64;  // items per workgroup of fg_factor_lane_kernel

// The tree sum (or max) of a group's per-lane values t[0..G) that the
// DPP butterflies of group_sum_d / group_max_d form (neighbours first).
// N = MM/4 entries; G <= N (uniform), a power of two.  Statically indexed.
template <int MODE, int N>
__device__ __forceinline__ double lane_tree(double (&t)[N], int G) {
#pragma unroll
    for (int w = 1; w < N; w *= 2) {
        if (w >= G) break;
#pragma unroll
        for (int p = 0; p + w < N; p += 2 * w) t[p] = MODE == kSum ? t[p] + t[p + w] : fmax(t[p], t[p + w]);
    }
    return t[0];
}

template <int MM, int MODE>
__global__ __launch_bounds__(kFgLane) void fg_factor_lane_kernel(FgArgs a) {
    const int lane = (int)threadIdx.x;
    const int item = a.items[blockIdx.x * kFgLane + lane];  // a * 3 + i, or -1
    // every run of items starts a workgroup with a real item
    const int first = __builtin_amdgcn_readfirstlane(a.items[blockIdx.x * kFgLane]);
    const int k = __builtin_amdgcn_readfirstlane(a.fac_type[first / 3]);
    const int i = first - 3 * (first / 3);
    const int M = a.M;
    const int G = lanes_for(M);
    const int n_oth = a.arity[k] - 1;
    const int j0 = i == 0 ? 1 : 0;
    const int j1 = i == 2 ? 1 : 2;
    const bool live = item >= 0;
    const int fa = live ? item / 3 : 0;
    const bool vec = (M & 3) == 0;  // rows of whole float4s
    const int* row = a.tptr + ((size_t)k * 3 + i) * (M + 1);
    // this lane's copies of the other slots' messages; the gathers below
    // index them with a wave-uniform label (relative register moves; two
    // arrays, each small enough to stay in registers)
    float n0[MM], n1[MM];
    double agg[2] = {1.0, 1.0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const float* src = a.n_vf + ((size_t)fa * 3 + (q ? j1 : j0)) * M;
        const bool use = live && q < n_oth;
        double t[MM / kLpl];
#pragma unroll
        for (int c = 0; c < MM / kLpl; ++c) {
            float v[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (use && c * kLpl < M) {
                if (vec) {
                    const v4f x = *reinterpret_cast<const v4f*>(src + c * kLpl);
                    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                } else {
#pragma unroll
                    for (int l = 0; l < kLpl; ++l)
                        if (c * kLpl + l < M) v[l] = src[c * kLpl + l];
                }
            }
#pragma unroll
            for (int l = 0; l < kLpl; ++l) (q ? n1 : n0)[c * kLpl + l] = v[l];
            t[c] = MODE == kSum ? ((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3])
                                : fmax(fmax((double)v[0], (double)v[1]), fmax((double)v[2], (double)v[3]));
        }
        if (q < n_oth) agg[q] = lane_tree<MODE, MM / kLpl>(t, G);
    }
    double base = (double)a.fbar[k] * agg[0];
    if (n_oth == 2) base *= agg[1];
    double u[MM];
#pragma unroll
    for (int x = 0; x < MM; ++x) {
        double acc = 0.0;  // labels beyond M count 0 in the normaliser
        if (x < M) {
            acc = base;
            const int e1 = row[x + 1];
#pragma unroll 4
            for (int e = row[x]; e < e1; ++e) {
                const int2 o = a.ent_o[e];
                double p = MODE == kSum ? a.ent_w[e] : (double)a.ent_f[e];
                p *= (double)n0[o.x];
                if (n_oth == 2) p *= (double)n1[o.y];
                acc = MODE == kSum ? acc + p : fmax(acc, p);
            }
        }
        u[x] = acc;
    }
    // normalise_d: each lane's 4 labels summed in order from 0, then the tree
    double t[MM / kLpl];
#pragma unroll
    for (int c = 0; c < MM / kLpl; ++c) {
        double z = 0.0;
#pragma unroll
        for (int l = 0; l < kLpl; ++l) z += u[c * kLpl + l];
        t[c] = z;
    }
    const double inv = recip_d(lane_tree<kSum, MM / kLpl>(t, G));
    if (!live) return;
    float* dst = a.m_fv + (size_t)item * M;
#pragma unroll
    for (int c = 0; c < MM / kLpl; ++c) {
        if (c * kLpl >= M) break;
        float m[kLpl];
#pragma unroll
        for (int l = 0; l < kLpl; ++l) m[l] = (float)(u[c * kLpl + l] * inv);
        if (vec) {
            *reinterpret_cast<v4f*>(dst + c * kLpl) = v4f{m[0], m[1], m[2], m[3]};
        } else {
#pragma unroll
            for (int l = 0; l < kLpl; ++l)
                if (c * kLpl + l < M) dst[c * kLpl + l] = m[l];
        }
    }
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
