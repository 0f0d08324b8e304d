// General sparse-compatible potentials (Sec. 4, Sec. 7) and the Eq. 10
// max-product fallback of the window potential: host-side tables,
// validation and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/bp.h"
#include "bp_general.hpp"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using namespace bpi;

namespace {

// Table sections, each 256-byte aligned: ptr, ent_x, ent_f, ent_w, mask.
struct TabLayout {
    size_t off[5];
    size_t total;
};

TabLayout layout(int n_types, int M, size_t entries_per_orientation) {
    const size_t mw = (size_t)(M + 31) / 32;
    const size_t e2 = 2 * entries_per_orientation;
    const size_t sz[5] = {(size_t)n_types * 2 * (M + 1) * sizeof(int), e2 * sizeof(int), e2 * sizeof(float),
                          e2 * sizeof(double), (size_t)n_types * 2 * M * mw * sizeof(unsigned)};
    TabLayout L;
    size_t o = 0;
    for (int i = 0; i < 5; ++i) {
        L.off[i] = o;
        o += bp_align_up(std::max<size_t>(sz[i], 1), 256);
    }
    L.total = o;
    for (int i = 0; i < 5; ++i) BP_ASSERT(L.off[i] % 256 == 0 && L.off[i] + sz[i] <= L.total);
    return L;
}

// One type in the caller's orientation: for each label y of the second node
// of a pair (right / bottom), the compatible labels x of the first node in
// ascending order, with f(x, y).
struct HostType {
    std::vector<int> ptr;  // [M + 1]
    std::vector<int> x;
    std::vector<float> f;
    float fbar;
};

// Host image of the tables for `types` and the launch scalars in G.
void build_image(bp_grid* G, const std::vector<HostType>& types, size_t entries, char* dev_dst) {
    const int M = G->M, nt = (int)types.size();
    const TabLayout L = layout(nt, M, entries);
    const int mw = (M + 31) / 32;
    G->gen_host.assign(L.total, 0);
    char* base = G->gen_host.data();
    int* ptr = reinterpret_cast<int*>(base + L.off[0]);
    int* ex = reinterpret_cast<int*>(base + L.off[1]);
    float* ef = reinterpret_cast<float*>(base + L.off[2]);
    double* ew = reinterpret_cast<double*>(base + L.off[3]);
    unsigned* mk = reinterpret_cast<unsigned*>(base + L.off[4]);
    int e = 0;
    int longest_eq10 = 0;
    for (int k = 0; k < nt; ++k) {
        const HostType& t = types[k];
        G->gen_fbar[k] = t.fbar;
        G->gen_fbar_d[k] = (double)t.fbar;
        G->gen_eq10[k] = 0;
        for (float f : t.f)
            if (f < t.fbar) G->gen_eq10[k] = 1;
        // orientation 0: messages to the right / down, target = second node's label
        // orientation 1: messages to the left / up, target = first node's label (the transpose)
        std::vector<std::vector<std::pair<int, float>>> rows[2];
        rows[0].resize(M);
        rows[1].resize(M);
        for (int y = 0; y < M; ++y)
            for (int q = t.ptr[y]; q < t.ptr[y + 1]; ++q) {
                rows[0][y].push_back({t.x[q], t.f[q]});
                rows[1][t.x[q]].push_back({y, t.f[q]});  // y ascending: each row stays sorted
            }
        for (int s = 0; s < 2; ++s) {
            const int ts = 2 * k + s;
            for (int y = 0; y < M; ++y) {
                ptr[ts * (M + 1) + y] = e;
                if (G->gen_eq10[k]) longest_eq10 = std::max(longest_eq10, (int)rows[s][y].size());
                for (auto& xf : rows[s][y]) {
                    ex[e] = xf.first;
                    ef[e] = xf.second;
                    ew[e] = (double)xf.second - (double)t.fbar;
                    mk[((size_t)ts * M + y) * mw + (xf.first >> 5)] |= 1u << (xf.first & 31);
                    ++e;
                }
            }
            ptr[ts * (M + 1) + M] = e;
        }
    }
    G->gen_types = nt;
    G->gen_mask_words = mw;
    G->gen_entries = (int)(2 * entries);
    G->gen_top_k = longest_eq10 > 0 ? longest_eq10 + 1 : 0;
    for (int i = 0; i < 5; ++i) G->gen_off[i] = L.off[i];
    G->gen_tab = dev_dst;
}

int upload_image(bp_grid* G) {
    hipError_t e = hipMemcpyAsync(G->gen_tab, G->gen_host.data(), G->gen_host.size(), hipMemcpyHostToDevice,
                                  G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "potential table upload");
}

// The host image is the source of an asynchronous copy: wait for any copy
// still reading it before it is rebuilt.
int drain(bp_grid* G) {
    hipError_t e = hipStreamSynchronize(G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // namespace

namespace bpi {

size_t window_table_bytes(int M) { return layout(1, M, (size_t)M * M).total; }

int build_window_tables(bp_grid* G) {
    if (G->win_tab_valid) return BP_OK;
    int st = drain(G);
    if (st) return st;
    HostType t;
    t.fbar = G->fbar;
    t.ptr.assign(G->M + 1, 0);
    for (int y = 0; y < G->M; ++y) {
        t.ptr[y] = (int)t.x.size();
        for (int x = std::max(0, y - G->T); x <= std::min(G->M - 1, y + G->T); ++x) {
            t.x.push_back(x);
            t.f.push_back(G->tab_f[x > y ? x - y : y - x]);  // the float32 table of the window kernel
        }
    }
    t.ptr[G->M] = (int)t.x.size();
    const size_t msg = 2 * bp_align_up(G->msg_floats() * sizeof(float), 256);
    build_image(G, {t}, t.x.size(), static_cast<char*>(G->ws) + msg);
    if ((st = upload_image(G))) return st;
    G->win_tab_valid = true;
    return BP_OK;
}

namespace {

bpk::GenArgs general_args(const bp_grid* G, const bpk::UpdateArgs& u) {
    bpk::GenArgs a;
    memset(&a, 0, sizeof a);
    a.u = u;
    a.type_h = G->general ? G->type_h : nullptr;
    a.type_v = G->general ? G->type_v : nullptr;
    a.ptr = reinterpret_cast<const int*>(G->gen_tab + G->gen_off[0]);
    a.ent_x = reinterpret_cast<const int*>(G->gen_tab + G->gen_off[1]);
    a.ent_f = reinterpret_cast<const float*>(G->gen_tab + G->gen_off[2]);
    a.ent_w = reinterpret_cast<const double*>(G->gen_tab + G->gen_off[3]);
    a.mask = reinterpret_cast<const unsigned*>(G->gen_tab + G->gen_off[4]);
    a.mask_words = G->gen_mask_words;
    a.n_entries = G->gen_entries;
    a.n_types = G->gen_types;
    a.top_k = G->gen_top_k;
    for (int k = 0; k < G->gen_types; ++k) {
        a.fbar[k] = G->gen_fbar[k];
        a.fbar_d[k] = G->gen_fbar_d[k];
        a.eq10[k] = G->gen_eq10[k];
    }
    return a;
}

}  // namespace

hipError_t launch_general_update(const bp_grid* G, const bpk::UpdateArgs& u, int kmode) {
    return bpk::launch_general(general_args(G, u), kmode, G->stream);
}

int iterate_general(bp_grid* G, int kmode, int n, int schedule) {
    if (schedule == BP_SCHED_SWEEP) {
        // one sweep = passes left, right, up, down; each axis's two passes
        // are independent and run as one launch (as in bp_iterate)
        for (int t = 0; t < n; ++t)
            for (int dir : {bpk::kLeft, bpk::kUp}) {
                bpk::UpdateArgs u = base_args(G, G->msg[G->cur], G->msg[G->cur], -1);
                u.dir = dir;
                u.both = 1;
                hipError_t e = bpk::launch_general_sweep(general_args(G, u), kmode, G->stream);
                if (e != hipSuccess) return hip_fail(e, "general sweep pass launch");
            }
        return BP_OK;
    }
    for (int t = 0; t < n; ++t) {
        const bpk::UpdateArgs u = schedule == BP_SCHED_SYNC
                                      ? base_args(G, G->msg[G->cur], G->msg[G->cur ^ 1], -1)
                                      : base_args(G, G->msg[G->cur], G->msg[G->cur], (int)(G->cb_pass & 1));
        hipError_t e = launch_general_update(G, u, kmode);
        if (e != hipSuccess) return hip_fail(e, "general update launch");
        if (schedule == BP_SCHED_SYNC) G->cur ^= 1;
        else G->cb_pass++;
    }
    return BP_OK;
}

}  // namespace bpi

namespace {

int check_types(const bp_grid* G, int32_t n_types, const bp_sparse_potential* types, size_t* entries) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called (it fixes M)");
    if (n_types < 1 || n_types > bpk::kMaxTypes || !types)
        return fail(BP_EINVAL, "n_types must be in [1, %d]", bpk::kMaxTypes);
    const int M = G->M;
    size_t total = 0;
    for (int k = 0; k < n_types; ++k) {
        const bp_sparse_potential& t = types[k];
        if (!t.col_ptr || (!t.row_idx && t.col_ptr[M] > 0) || (!t.val && t.col_ptr[M] > 0))
            return fail(BP_EINVAL, "type %d: null table", k);
        if (!std::isfinite(t.fbar) || t.fbar < 0.0f) return fail(BP_EINVAL, "type %d: fbar must be finite and >= 0", k);
        if (t.col_ptr[0] != 0) return fail(BP_EINVAL, "type %d: col_ptr[0] must be 0", k);
        for (int y = 0; y < M; ++y) {
            if (t.col_ptr[y + 1] < t.col_ptr[y] || t.col_ptr[y + 1] - t.col_ptr[y] > M)
                return fail(BP_EINVAL, "type %d: col_ptr not non-decreasing at %d", k, y);
            for (int q = t.col_ptr[y]; q < t.col_ptr[y + 1]; ++q) {
                const int x = t.row_idx[q];
                if (x < 0 || x >= M) return fail(BP_EINVAL, "type %d: label %d out of range", k, x);
                if (q > t.col_ptr[y] && x <= t.row_idx[q - 1])
                    return fail(BP_EINVAL, "type %d: labels of column %d not strictly increasing", k, y);
                if (!std::isfinite(t.val[q]) || t.val[q] < 0.0f)
                    return fail(BP_EINVAL, "type %d: values must be finite and >= 0", k);
            }
        }
        total += (size_t)t.col_ptr[M];
    }
    *entries = total;
    return BP_OK;
}

int check_type_map(const bp_grid* G, const uint8_t* map_dev, size_t n, int n_types, const char* what) {
    if (!map_dev || n == 0) return BP_OK;
    std::vector<uint8_t> h(n);
    hipError_t e = hipMemcpy(h.data(), map_dev, n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, what);
    for (uint8_t v : h)
        if (v >= n_types) return fail(BP_EINVAL, "%s: type %d >= n_types %d", what, (int)v, n_types);
    return BP_OK;
}

}  // namespace

extern "C" {

int64_t bp_sparse_table_bytes(const bp_grid* G, int32_t n_types, const bp_sparse_potential* types) {
    size_t entries = 0;
    int st = check_types(G, n_types, types, &entries);
    if (st) return st;
    return (int64_t)layout(n_types, G->M, entries).total;
}

int bp_set_sparse_potentials(bp_grid* G, int32_t n_types, const bp_sparse_potential* types, void* table_dev,
                             int64_t table_bytes, const uint8_t* type_h_dev, const uint8_t* type_v_dev) {
    size_t entries = 0;
    int st = check_types(G, n_types, types, &entries);
    if (st) return st;
    invalidate_grad(G);
    if (!table_dev || reinterpret_cast<uintptr_t>(table_dev) % 256)
        return fail(BP_EINVAL, "table buffer null or not 256-byte aligned");
    const size_t need = layout(n_types, G->M, entries).total;
    if (table_bytes < (int64_t)need)
        return fail(BP_ENOMEM, "table buffer %lld bytes < %zu needed", (long long)table_bytes, need);
    if ((st = with_device(G))) return st;
    if ((st = check_type_map(G, type_h_dev, (size_t)G->H * (G->W - 1), n_types, "horizontal type map"))) return st;
    if ((st = check_type_map(G, type_v_dev, (size_t)(G->H - 1) * G->W, n_types, "vertical type map"))) return st;
    if ((st = drain(G))) return st;
    std::vector<HostType> ht(n_types);
    for (int k = 0; k < n_types; ++k) {
        const bp_sparse_potential& t = types[k];
        const int nnz = t.col_ptr[G->M];
        ht[k].ptr.assign(t.col_ptr, t.col_ptr + G->M + 1);
        ht[k].x.assign(t.row_idx, t.row_idx + nnz);
        ht[k].f.assign(t.val, t.val + nnz);
        ht[k].fbar = t.fbar;
    }
    build_image(G, ht, entries, static_cast<char*>(table_dev));
    if ((st = upload_image(G))) return st;
    G->type_h = type_h_dev;
    G->type_v = type_v_dev;
    G->general = true;
    G->win_tab_valid = false;
    return BP_OK;
}

}  // extern "C"
