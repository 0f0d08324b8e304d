// Factor-graph BP with sparse-compatible higher-order factors (Sec. 7):
// host-side graph, tables, workspace and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/bp.h"
#include "bp_factor.hpp"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using namespace bpi;

namespace {

struct Tables {  // one CSR set (sparse, or the complete dense lists)
    std::vector<int> tptr;            // [n_types][3][M + 1]
    std::vector<int2> ent_o;
    std::vector<float> ent_f;
    std::vector<double> ent_w;
    std::vector<int2> ent_s;          // each row's other-slot labels sorted by (a, b)
    int top[bpk::kFgMaxTypes][3][2] = {};  // split form's top-list lengths per type and slot
    int most_entries = 0;             // largest (type, slot) table: the entries a workgroup stages
    size_t off[5] = {};               // device offsets: tptr, ent_o, ent_f, ent_w, ent_s
};

}  // namespace

struct bp_fgraph {
    int dev = 0;
    hipStream_t stream = nullptr;
    int n_vars = 0, M = 0, n_factors = 0, n_types = 0;
    std::vector<int> fac_type, var_ptr, var_adj;
    std::vector<int> items;           // factor messages grouped by (type, slot), runs padded to workgroups
    int arity[bpk::kFgMaxTypes] = {};
    float fbar[bpk::kFgMaxTypes] = {};
    bool eq11_ok[bpk::kFgMaxTypes] = {};  // every compatible f >= fbar
    Tables sparse, dense;
    bool has_dense = false;
    // device
    char* ws = nullptr;
    int64_t ws_bytes = 0;
    size_t off_type = 0, off_vptr = 0, off_vadj = 0, off_items = 0, off_m = 0, off_n = 0, total = 0;
    std::vector<char> image;          // host source of the table upload
    const float* g = nullptr;
};

namespace {

// Per type and slot i, the tuples grouped by their label at i, tuple order
// kept; entries hold the other slots' labels in slot order.
void build_tables(bp_fgraph* F, const std::vector<std::vector<int>>& tup, const std::vector<std::vector<float>>& val,
                  const float* fbar, Tables& T) {
    const int M = F->M;
    T.tptr.assign((size_t)F->n_types * 3 * (M + 1), 0);
    T.ent_o.clear();
    T.ent_f.clear();
    T.ent_w.clear();
    T.ent_s.clear();
    T.most_entries = 0;
    for (int k = 0; k < F->n_types; ++k) {
        const int K = F->arity[k];
        const size_t C = val[k].size();
        for (int i = 0; i < 3; ++i) {
            int* row = T.tptr.data() + ((size_t)k * 3 + i) * (M + 1);
            if (i >= K) {
                for (int x = 0; x <= M; ++x) row[x] = (int)T.ent_o.size();
                continue;
            }
            std::vector<std::vector<size_t>> by(M);
            for (size_t c = 0; c < C; ++c) by[tup[k][c * K + i]].push_back(c);
            for (int x = 0; x < M; ++x) {
                row[x] = (int)T.ent_o.size();
                for (size_t c : by[x]) {
                    int o[2] = {-1, -1}, q = 0;
                    for (int j = 0; j < K; ++j)
                        if (j != i) o[q++] = tup[k][c * K + j];
                    T.ent_o.push_back(make_int2(o[0], o[1]));
                    T.ent_f.push_back(val[k][c]);
                    T.ent_w.push_back((double)val[k][c] - (double)fbar[k]);
                }
            }
            row[M] = (int)T.ent_o.size();
            // Sorted copy for the split form's membership tests, and its
            // top-list lengths: one more than the most first labels listed
            // in a row (pairs: the most entries), and one more than the
            // longest run of one first label; at most M.
            int most_a = 0, most_run = 0;
            for (int x = 0; x < M; ++x) {
                std::vector<int2> r(T.ent_o.begin() + row[x], T.ent_o.begin() + row[x + 1]);
                std::sort(r.begin(), r.end(), [](int2 p, int2 q) { return p.x != q.x ? p.x < q.x : p.y < q.y; });
                int distinct = 0;
                for (size_t e = 0; e < r.size();) {
                    size_t f = e;
                    while (f < r.size() && r[f].x == r[e].x) ++f;
                    ++distinct;
                    most_run = std::max(most_run, (int)(f - e));
                    e = f;
                }
                most_a = std::max(most_a, distinct);
                T.ent_s.insert(T.ent_s.end(), r.begin(), r.end());
            }
            T.top[k][i][0] = std::min(M, most_a + 1);
            T.top[k][i][1] = K == 3 ? std::min(M, most_run + 1) : 0;
            T.most_entries = std::max(T.most_entries, row[M] - row[0]);
        }
    }
}

size_t place(size_t& off, size_t bytes) {
    const size_t at = off;
    off += bp_align_up(std::max<size_t>(bytes, 1), 256);
    BP_ASSERT(at % 256 == 0 && off >= at + bytes);
    return at;
}

void layout_tables(Tables& T, size_t& off) {
    T.off[0] = place(off, T.tptr.size() * sizeof(int));
    T.off[1] = place(off, T.ent_o.size() * sizeof(int2));
    T.off[2] = place(off, T.ent_f.size() * sizeof(float));
    T.off[3] = place(off, T.ent_w.size() * sizeof(double));
    T.off[4] = place(off, T.ent_s.size() * sizeof(int2));
}

void copy_tables(const Tables& T, char* img) {
    memcpy(img + T.off[0], T.tptr.data(), T.tptr.size() * sizeof(int));
    memcpy(img + T.off[1], T.ent_o.data(), T.ent_o.size() * sizeof(int2));
    memcpy(img + T.off[2], T.ent_f.data(), T.ent_f.size() * sizeof(float));
    memcpy(img + T.off[3], T.ent_w.data(), T.ent_w.size() * sizeof(double));
    memcpy(img + T.off[4], T.ent_s.data(), T.ent_s.size() * sizeof(int2));
}

bpk::FgArgs args(const bp_fgraph* F, bool dense) {
    bpk::FgArgs a;
    memset(&a, 0, sizeof a);
    const Tables& T = dense ? F->dense : F->sparse;
    a.g = F->g;
    a.var_ptr = reinterpret_cast<const int*>(F->ws + F->off_vptr);
    a.var_adj = reinterpret_cast<const int*>(F->ws + F->off_vadj);
    a.fac_type = reinterpret_cast<const int*>(F->ws + F->off_type);
    a.tptr = reinterpret_cast<const int*>(F->ws + T.off[0]);
    a.ent_o = reinterpret_cast<const int2*>(F->ws + T.off[1]);
    a.ent_f = reinterpret_cast<const float*>(F->ws + T.off[2]);
    a.ent_w = reinterpret_cast<const double*>(F->ws + T.off[3]);
    a.ent_s = reinterpret_cast<const int2*>(F->ws + T.off[4]);
    a.items = reinterpret_cast<const int*>(F->ws + F->off_items);
    a.n_items = (int)F->items.size();
    a.m_fv = reinterpret_cast<float*>(F->ws + F->off_m);
    a.n_vf = reinterpret_cast<float*>(F->ws + F->off_n);
    a.n_vars = F->n_vars;
    a.n_factors = F->n_factors;
    a.M = F->M;
    for (int k = 0; k < F->n_types; ++k) {
        a.arity[k] = F->arity[k];
        a.fbar[k] = dense ? 0.0f : F->fbar[k];
        a.eq10[k] = !dense && !F->eq11_ok[k];  // the complete lists have fbar = 0 <= every f
        for (int i = 0; i < 3; ++i)
            for (int q = 0; q < 2; ++q) a.top[k][i][q] = T.top[k][i][q];
    }
    return a;
}

int ready(const bp_fgraph* F) {
    if (!F) return fail(BP_EINVAL, "null factor-graph handle");
    if (!F->ws) return fail(BP_ESTATE, "no workspace attached");
    return BP_OK;
}

int set_dev(const bp_fgraph* F) {
    hipError_t e = hipSetDevice(F->dev);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipSetDevice");
}

}  // namespace

extern "C" {

int bp_fg_init(bp_fgraph** out, int32_t n_vars, int32_t M, int32_t n_factors, const int32_t* factor_vars,
               const int32_t* factor_type, int32_t n_types, const bp_factor_type* types, int32_t dense_tables,
               void* hip_stream) {
    if (!out) return fail(BP_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (n_vars < 1 || M < 1 || M > BP_MAX_LABELS || n_factors < 0 || (n_factors > 0 && (!factor_vars || !factor_type)))
        return fail(BP_EINVAL, "bad sizes (n_vars >= 1, 1 <= M <= %d, n_factors >= 0)", BP_MAX_LABELS);
    if (n_types < 1 || n_types > bpk::kFgMaxTypes || !types)
        return fail(BP_EINVAL, "n_types must be in [1, %d]", bpk::kFgMaxTypes);
    if ((int64_t)n_factors * 3 * M >= (int64_t(1) << 31)) return fail(BP_EINVAL, "too many factor messages");
    bp_fgraph* F = new (std::nothrow) bp_fgraph();
    if (!F) return fail(BP_ENOMEM, "host allocation failed");
    F->stream = static_cast<hipStream_t>(hip_stream);
    F->n_vars = n_vars;
    F->M = M;
    F->n_factors = n_factors;
    F->n_types = n_types;
    std::vector<std::vector<int>> tup(n_types);
    std::vector<std::vector<float>> val(n_types);
    for (int k = 0; k < n_types; ++k) {
        const bp_factor_type& t = types[k];
        if (t.arity != 2 && t.arity != 3) { delete F; return fail(BP_EINVAL, "type %d: arity must be 2 or 3", k); }
        if (t.n_tuples < 0 || (t.n_tuples > 0 && (!t.tuples || !t.val))) {
            delete F;
            return fail(BP_EINVAL, "type %d: bad tuple list", k);
        }
        if (!std::isfinite(t.fbar) || t.fbar < 0.0f) { delete F; return fail(BP_EINVAL, "type %d: bad fbar", k); }
        F->arity[k] = t.arity;
        F->fbar[k] = t.fbar;
        F->eq11_ok[k] = true;
        std::unordered_set<int64_t> seen;
        for (int c = 0; c < t.n_tuples; ++c) {
            int64_t key = 0;
            for (int j = 0; j < t.arity; ++j) {
                const int x = t.tuples[(size_t)c * t.arity + j];
                if (x < 0 || x >= M) { delete F; return fail(BP_EINVAL, "type %d: label %d out of range", k, x); }
                key = key * M + x;
            }
            if (!seen.insert(key).second) { delete F; return fail(BP_EINVAL, "type %d: duplicate tuple %d", k, c); }
            if (!std::isfinite(t.val[c]) || t.val[c] < 0.0f) {
                delete F;
                return fail(BP_EINVAL, "type %d: values must be finite and >= 0", k);
            }
            if (t.val[c] < t.fbar) F->eq11_ok[k] = false;
        }
        tup[k].assign(t.tuples, t.tuples + (size_t)t.n_tuples * t.arity);
        val[k].assign(t.val, t.val + t.n_tuples);
    }
    // variables' incident slots, in factor order
    std::vector<std::vector<int>> adj(n_vars);
    F->fac_type.assign(factor_type, factor_type + n_factors);
    for (int a = 0; a < n_factors; ++a) {
        const int k = factor_type[a];
        if (k < 0 || k >= n_types) { delete F; return fail(BP_EINVAL, "factor %d: bad type %d", a, k); }
        for (int i = 0; i < F->arity[k]; ++i) {
            const int v = factor_vars[(size_t)a * 3 + i];
            if (v < 0 || v >= n_vars) { delete F; return fail(BP_EINVAL, "factor %d: bad variable %d", a, v); }
            for (int j = 0; j < i; ++j)
                if (factor_vars[(size_t)a * 3 + j] == v) { delete F; return fail(BP_EINVAL, "factor %d: repeated variable", a); }
            adj[v].push_back(a * 3 + i);
        }
    }
    // Factor messages grouped by (type, slot), factor order inside a group,
    // each run padded with -1 to a multiple of kFgLane items: whole
    // workgroups of either factor kernel (kFgLane items, or kBlock/G).
    const int rpb = bpk::kFgLane;
    for (int k = 0; k < n_types; ++k)
        for (int i = 0; i < F->arity[k]; ++i) {
            size_t n = 0;
            for (int a = 0; a < n_factors; ++a)
                if (factor_type[a] == k) {
                    F->items.push_back(a * 3 + i);
                    ++n;
                }
            while (n % rpb) {
                F->items.push_back(-1);
                ++n;
            }
        }
    F->var_ptr.assign(n_vars + 1, 0);
    for (int v = 0; v < n_vars; ++v) {
        F->var_ptr[v + 1] = F->var_ptr[v] + (int)adj[v].size();
        F->var_adj.insert(F->var_adj.end(), adj[v].begin(), adj[v].end());
    }
    build_tables(F, tup, val, F->fbar, F->sparse);
    if (dense_tables) {
        // every tuple listed, with its table value (fbar outside C); the
        // fbar term of the update is then zero
        std::vector<std::vector<int>> dt(n_types);
        std::vector<std::vector<float>> dv(n_types);
        float zero[bpk::kFgMaxTypes] = {};
        for (int k = 0; k < n_types; ++k) {
            const int K = F->arity[k];
            size_t total = 1;
            for (int j = 0; j < K; ++j) total *= (size_t)M;
            if (total > (size_t)1 << 24) { delete F; return fail(BP_EUNSUPPORTED, "dense tables above 2^24 tuples"); }
            std::vector<float> table(total, F->fbar[k]);
            for (size_t c = 0; c < val[k].size(); ++c) {
                size_t key = 0;
                for (int j = 0; j < K; ++j) key = key * M + tup[k][c * K + j];
                table[key] = val[k][c];
            }
            for (size_t key = 0; key < total; ++key) {
                size_t r = key;
                int lab[3];
                for (int j = K - 1; j >= 0; --j) { lab[j] = (int)(r % M); r /= M; }
                for (int j = 0; j < K; ++j) dt[k].push_back(lab[j]);
                dv[k].push_back(table[key]);
            }
        }
        build_tables(F, dt, dv, zero, F->dense);
        F->has_dense = true;
    }
    size_t off = 0;
    F->off_type = place(off, (size_t)n_factors * sizeof(int));
    F->off_vptr = place(off, (size_t)(n_vars + 1) * sizeof(int));
    F->off_vadj = place(off, F->var_adj.size() * sizeof(int));
    F->off_items = place(off, F->items.size() * sizeof(int));
    layout_tables(F->sparse, off);
    if (F->has_dense) layout_tables(F->dense, off);
    const size_t tables_end = off;
    F->off_m = place(off, (size_t)n_factors * 3 * M * sizeof(float));
    F->off_n = place(off, (size_t)n_factors * 3 * M * sizeof(float));
    F->total = off;
    F->image.assign(tables_end, 0);
    memcpy(F->image.data() + F->off_type, F->fac_type.data(), F->fac_type.size() * sizeof(int));
    memcpy(F->image.data() + F->off_vptr, F->var_ptr.data(), F->var_ptr.size() * sizeof(int));
    memcpy(F->image.data() + F->off_vadj, F->var_adj.data(), F->var_adj.size() * sizeof(int));
    memcpy(F->image.data() + F->off_items, F->items.data(), F->items.size() * sizeof(int));
    copy_tables(F->sparse, F->image.data());
    if (F->has_dense) copy_tables(F->dense, F->image.data());
    BP_ASSERT(F->off_items + F->items.size() * sizeof(int) <= tables_end && tables_end <= F->off_m);
    BP_ASSERT(F->off_n + (size_t)n_factors * 3 * M * sizeof(float) <= F->total);
    int dev = -1;  // after the host-side build: argument errors are reported as such without a device
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) {
        delete F;
        return hip_fail(he, "hipGetDevice");
    }
    F->dev = dev;
    *out = F;
    return BP_OK;
}

int64_t bp_fg_workspace_bytes(const bp_fgraph* F) {
    if (!F) return fail(BP_EINVAL, "null factor-graph handle");
    return (int64_t)F->total;
}

int bp_fg_attach_workspace(bp_fgraph* F, void* dev_ptr, int64_t bytes) {
    if (!F) return fail(BP_EINVAL, "null factor-graph handle");
    if (!dev_ptr || reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(BP_EINVAL, "workspace null or misaligned");
    if (bytes < (int64_t)F->total) return fail(BP_ENOMEM, "workspace %lld bytes < %zu needed", (long long)bytes, F->total);
    int st = set_dev(F);
    if (st) return st;
    hipError_t e = hipStreamSynchronize(F->stream);  // a previous upload may still read the image
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    F->ws = static_cast<char*>(dev_ptr);
    F->ws_bytes = bytes;
    e = hipMemcpyAsync(F->ws, F->image.data(), F->image.size(), hipMemcpyHostToDevice, F->stream);
    if (e != hipSuccess) return hip_fail(e, "factor-graph table upload");
    return bp_fg_reset_messages(F);
}

int bp_fg_set_unary(bp_fgraph* F, const float* g_dev) {
    if (!F) return fail(BP_EINVAL, "null factor-graph handle");
    if (!g_dev || reinterpret_cast<uintptr_t>(g_dev) % 16) return fail(BP_EINVAL, "unary null or not 16-byte aligned");
    F->g = g_dev;
    return BP_OK;
}

int bp_fg_set_stream(bp_fgraph* F, void* hip_stream) {
    if (!F) return fail(BP_EINVAL, "null factor-graph handle");
    F->stream = static_cast<hipStream_t>(hip_stream);
    return BP_OK;
}

int bp_fg_reset_messages(bp_fgraph* F) {
    int st = ready(F);
    if (st) return st;
    if ((st = set_dev(F))) return st;
    const size_t n = (size_t)F->n_factors * 3 * F->M;
    for (size_t o : {F->off_m, F->off_n}) {
        hipError_t e = bpk::launch_fill(reinterpret_cast<float*>(F->ws + o), n, 1.0f / (float)F->M, F->stream);
        if (e != hipSuccess) return hip_fail(e, "factor-graph message reset");
    }
    return BP_OK;
}

int bp_fg_iterate(bp_fgraph* F, int32_t mode, int32_t n_iters, int32_t dense) {
    bpi::TraceRange tr("bp_fg_iterate");
    int st = ready(F);
    if (st) return st;
    if (!F->g) return fail(BP_ESTATE, "bp_fg_set_unary has not been called");
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (n_iters < 0) return fail(BP_EINVAL, "n_iters < 0");
    if (dense && !F->has_dense) return fail(BP_ESTATE, "dense tables were not built (bp_fg_init dense_tables = 0)");
    bool split = false;  // max-product with some f < fbar: the split form (Eq. 10's analogue)
    if (mode == BP_MAX_PRODUCT && !dense)
        for (int k = 0; k < F->n_types; ++k)
            if (!F->eq11_ok[k]) {
                split = true;
                for (int i = 0; i < F->arity[k]; ++i)
                    if (F->sparse.top[k][i][0] > bpk::kFgTop || F->sparse.top[k][i][1] > bpk::kFgTop)
                        return fail(BP_EUNSUPPORTED,
                                    "type %d: the split form needs at most %d listed labels per slot and label",
                                    k, bpk::kFgTop - 1);
            }
    if ((st = set_dev(F))) return st;
    const bpk::FgArgs a = args(F, dense != 0);
    for (int t = 0; t < n_iters; ++t) {
        hipError_t e = bpk::launch_fg_iteration(a, mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax, split,
                                                dense ? F->dense.most_entries : F->sparse.most_entries, F->stream);
        if (e != hipSuccess) return hip_fail(e, "factor-graph launch");
    }
    return BP_OK;
}

int bp_fg_beliefs(bp_fgraph* F, float* beliefs_dev, int32_t* labels_dev) {
    int st = ready(F);
    if (st) return st;
    if (!F->g) return fail(BP_ESTATE, "bp_fg_set_unary has not been called");
    if (!beliefs_dev && !labels_dev) return fail(BP_EINVAL, "no output");
    if (beliefs_dev && reinterpret_cast<uintptr_t>(beliefs_dev) % 16)
        return fail(BP_EINVAL, "beliefs output not 16-byte aligned");
    if ((st = set_dev(F))) return st;
    hipError_t e = bpk::launch_fg_beliefs(args(F, false), beliefs_dev, labels_dev, F->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "factor-graph readout");
}

int bp_fg_get_messages(const bp_fgraph* F, float* m_dev, float* n_dev) {
    int st = ready(F);
    if (st) return st;
    if ((st = set_dev(F))) return st;
    const size_t bytes = (size_t)F->n_factors * 3 * F->M * sizeof(float);
    if (m_dev) {
        hipError_t e = hipMemcpyAsync(m_dev, F->ws + F->off_m, bytes, hipMemcpyDeviceToDevice, F->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    if (n_dev) {
        hipError_t e = hipMemcpyAsync(n_dev, F->ws + F->off_n, bytes, hipMemcpyDeviceToDevice, F->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return BP_OK;
}

int bp_fg_destroy(bp_fgraph* F) {
    delete F;
    return BP_OK;
}

}  // extern "C"

namespace bpk {
namespace {

// The factor kernel stages its table in LDS when the largest (type, slot)
// table fits (most_entries <= fg_stage_entries).
template <int G, int MODE, bool SPLIT>
hipError_t go_iteration(const FgArgs& a, int most_entries, hipStream_t s) {
    constexpr int RPB = kBlock / G;
    constexpr bool kTops = SPLIT && MODE == kMax;
    if (a.n_vars > 0) {
        hipLaunchKernelGGL((fg_var_kernel<G>), dim3((a.n_vars + RPB - 1) / RPB), dim3(kBlock), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.n_items > 0) {
        if constexpr (!kTops && G <= 8) {
            // M <= 32 outside the split form: one message per lane
            const dim3 grid((unsigned)(a.n_items / kFgLane));
            if (a.M <= 16) hipLaunchKernelGGL((fg_factor_lane_kernel<16, MODE>), grid, dim3(kFgLane), 0, s, a);
            else hipLaunchKernelGGL((fg_factor_lane_kernel<32, MODE>), grid, dim3(kFgLane), 0, s, a);
            return hipGetLastError();
        }
        const unsigned blocks = (unsigned)(a.n_items / RPB);
        if ((size_t)most_entries <= fg_stage_entries(G, kTops))
            hipLaunchKernelGGL((fg_factor_kernel<G, MODE, SPLIT, true>), dim3(blocks), dim3(kBlock),
                               fg_lds_bytes(G, kTops) + (size_t)most_entries * (sizeof(double) + sizeof(int2)), s, a);
        else
            hipLaunchKernelGGL((fg_factor_kernel<G, MODE, SPLIT, false>), dim3(blocks), dim3(kBlock),
                               fg_lds_bytes(G, kTops), s, a);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <int G>
hipError_t go_beliefs(const FgArgs& a, float* b, int* lab, hipStream_t s) {
    constexpr int RPB = kBlock / G;
    hipLaunchKernelGGL((fg_belief_kernel<G>), dim3((a.n_vars + RPB - 1) / RPB), dim3(kBlock), 0, s, a, b, lab);
    return hipGetLastError();
}

template <int G>
hipError_t iteration_g(const FgArgs& a, int mode, bool split, int most_entries, hipStream_t s) {
    if (mode == kSum) return go_iteration<G, kSum, false>(a, most_entries, s);
    return split ? go_iteration<G, kMax, true>(a, most_entries, s) : go_iteration<G, kMax, false>(a, most_entries, s);
}

}  // namespace

hipError_t launch_fg_iteration(const FgArgs& a, int mode, bool split, int most_entries, hipStream_t s) {
    switch (lanes_for(a.M)) {
        case 4: return iteration_g<4>(a, mode, split, most_entries, s);
        case 8: return iteration_g<8>(a, mode, split, most_entries, s);
        case 16: return iteration_g<16>(a, mode, split, most_entries, s);
        case 32: return iteration_g<32>(a, mode, split, most_entries, s);
        default: return iteration_g<64>(a, mode, split, most_entries, s);
    }
}

hipError_t launch_fg_beliefs(const FgArgs& a, float* b, int* lab, hipStream_t s) {
    switch (lanes_for(a.M)) {
        case 4: return go_beliefs<4>(a, b, lab, s);
        case 8: return go_beliefs<8>(a, b, lab, s);
        case 16: return go_beliefs<16>(a, b, lab, s);
        case 32: return go_beliefs<32>(a, b, lab, s);
        default: return go_beliefs<64>(a, b, lab, s);
    }
}

}  // namespace bpk
