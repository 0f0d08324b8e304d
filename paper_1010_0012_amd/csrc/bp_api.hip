// C ABI of the grid BP library: handle state, argument and call-order checks,
// potential tables, workspace carving and kernel dispatch.
#include <dlfcn.h>

#include <algorithm>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bp.h"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using bpk::UpdateArgs;

namespace bpi {

thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(BP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Every call that changes the message state, the potential or the unary
// invalidates the checkpoints of a previous bp_forward_ckpt.
void invalidate_grad(bp_grid* G) { G->grad_ready = false; }

// f(d) = exp(-alpha d) in double; float32 tables for max-product and the
// float32 paths, the double window for sum-product.
void build_tables(bp_grid* G) {
    G->fbar_d = G->fbar_tied ? std::exp(-(double)G->alpha * G->T) : (double)G->fbar;
    for (int d = 0; d < bpk::kMaxTab; ++d) {
        const bool in = d <= G->T;
        const double f = std::exp(-(double)G->alpha * d);
        G->tab_f[d] = in ? (float)f : 0.0f;
        G->tab_w[d] = in ? (float)(f - (double)G->fbar) : 0.0f;
        if (d < bpk::kDTab) G->tab_wd[d] = in ? f - G->fbar_d : 0.0;
    }
}

bool max_product_ok(const bp_grid* G) {
    for (int d = 0; d <= G->T; ++d)
        if (!(G->tab_f[d] >= G->fbar)) return false;
    return true;
}

UpdateArgs base_args(const bp_grid* G, const float* in, float* out, int colour) {
    UpdateArgs a;
    memset(&a, 0, sizeof a);
    a.g = G->g;
    a.in = in;
    a.out = out;
    a.H = G->H;
    a.W = G->W;
    a.M = G->M;
    a.N = G->N;
    a.colour = colour;
    a.half_w = (G->W + 1) / 2;
    a.n_slots = colour < 0 ? G->N : G->H * a.half_w;
    a.T = G->T;
    a.fbar = G->fbar;
    a.fbar_d = G->fbar_d;
    a.alpha_d = (double)G->alpha;
    memcpy(a.dtab, G->tab_wd, sizeof a.dtab);
    a.pair_layout = G->pair_layout;
    a.pair_cap = G->pair_cap;
    return a;
}

int check_ready(const bp_grid* G) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    if (!G->ws) return fail(BP_ESTATE, "no workspace attached");
    if (!G->g) return fail(BP_ESTATE, "bp_set_unary has not been called");
    return BP_OK;
}

int with_device(const bp_grid* G) {
    hipError_t e = hipSetDevice(G->dev);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipSetDevice");
}

// n synchronous iterations (ping-pong), n checkerboard passes or n
// directional sweeps (both in place) of the sparse or dense update.
int iterate(bp_grid* G, int mode, int n, int schedule, bool dense) {
    int st = check_ready(G);
    if (st) return st;
    invalidate_grad(G);
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (schedule != BP_SCHED_SYNC && schedule != BP_SCHED_CHECKERBOARD && schedule != BP_SCHED_SWEEP)
        return fail(BP_EINVAL, "bad schedule %d", schedule);
    if (n < 0) return fail(BP_EINVAL, "n_iters < 0");
    const int kmode = mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax;
    // Max-product of the window potential when fbar exceeds f somewhere
    // (Eq. 11 does not hold; Eq. 10 does) runs the window kernels' Eq. 10
    // form where a register window is compiled, else the general kernel on
    // the window's tables; general sparse potentials run the general kernel.
    const bool eq10 = !G->general && mode == BP_MAX_PRODUCT && !max_product_ok(G) && !dense;
    const bool eq10_general = eq10 && bpk::sparse_variant_tw(G->M, G->T) < 0;
    if (G->general || eq10_general) {
        if (dense) return fail(BP_EUNSUPPORTED, "the dense kernel takes the truncated-linear potential only");
        if ((st = with_device(G))) return st;
        if (eq10_general && (st = build_window_tables(G))) return st;
        return iterate_general(G, kmode, n, schedule);
    }
    if (dense && G->M > 128) return fail(BP_EUNSUPPORTED, "dense kernel supports M <= 128");
    if (dense) {
        int max_lds = 0;
        hipError_t e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, G->dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        const int km = mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax;
        const size_t need = schedule == BP_SCHED_SWEEP ? bpk::sweep_dense_lds_need(G->M, km)
                                                       : bpk::dense_lds_need(G->M, km);
        if (need > (size_t)max_lds)
            return fail(BP_EUNSUPPORTED, "dense kernel needs %zu bytes of LDS per workgroup, device allows %d",
                        need, max_lds);
    }
    if ((st = with_device(G))) return st;
    // sparse sum uses w(d) = f(d) - fbar; sparse max and dense use f(d)
    const float* tab = (!dense && kmode == bpk::kSum) ? G->tab_w : G->tab_f;
    // float32 arithmetic (BP_ARITH_F32) where it is compiled: sum-product of
    // the window potential with fbar > 0 (every message entry then stays at
    // or above fbar/M, so h cannot underflow), any schedule, a register
    // window, full label rows (M = 4G), inbox planes below 2^32 bytes
    const bool f32 = G->arith_f32 && kmode == bpk::kSum && !dense && G->fbar > 0.0f &&
                     bpk::sparse_variant_tw(G->M, G->T) >= 0 && G->M == 4 * bpk::lanes_for(G->M) &&
                     (uint64_t)G->N * G->M * sizeof(float) < (uint64_t(1) << 32);
    const int kupd = f32 ? bpk::kSumF32 : kmode;
    if (schedule == BP_SCHED_SWEEP) {
        // One sweep = passes with messages travelling left, right, up, down.
        // The left and right passes are independent (each reads the up and
        // down planes and writes its own plane), as are up and down, so each
        // axis runs as one launch of both passes: the same result as four.
        for (int t = 0; t < n; ++t) {
            for (int dir : {bpk::kLeft, bpk::kUp}) {
                UpdateArgs a = base_args(G, G->msg[G->cur], G->msg[G->cur], -1);
                a.dir = dir;
                a.both = 1;
                a.eq10 = eq10;
                memcpy(a.tab, tab, sizeof a.tab);
                hipError_t e = bpk::launch_sweep(a, kupd, dense, G->stream);
                if (e != hipSuccess) return hip_fail(e, "sweep pass launch");
            }
        }
        return BP_OK;
    }
    // Iterations (sync) or passes (checkerboard) in pairs: one launch for two
    // (the same bits as two single launches), then a single launch for an
    // odd remainder.  A checkerboard pair writes the other buffer in full, so
    // it flips the current buffer; single passes stay in place.
    if (!dense && !eq10 && G->fuse_sync && bpk::sparse2_supported(G->M, G->T)) {
        for (; n >= 2; n -= 2) {
            UpdateArgs a;
            if (schedule == BP_SCHED_SYNC) {
                a = base_args(G, G->msg[G->cur], G->msg[G->cur ^ 1], -1);
            } else {
                // passes of colours c, 1 - c: the launch runs the colour 1 - c senders
                a = base_args(G, G->msg[G->cur], G->msg[G->cur ^ 1], (int)((G->cb_pass + 1) & 1));
                a.mid = G->msg[G->cur ^ 1];
            }
            memcpy(a.tab, tab, sizeof a.tab);
            hipError_t e = bpk::launch_sparse2(a, kupd, G->stream);
            if (e != hipSuccess) return hip_fail(e, "fused sparse update launch");
            G->cur ^= 1;
            if (schedule == BP_SCHED_CHECKERBOARD) G->cb_pass += 2;
        }
    }
    for (int t = 0; t < n; ++t) {
        UpdateArgs a;
        if (schedule == BP_SCHED_SYNC) {
            a = base_args(G, G->msg[G->cur], G->msg[G->cur ^ 1], -1);
        } else {
            a = base_args(G, G->msg[G->cur], G->msg[G->cur], (int)(G->cb_pass & 1));
        }
        memcpy(a.tab, tab, sizeof a.tab);
        a.eq10 = eq10;
        hipError_t e = dense ? bpk::launch_dense(a, kmode, G->stream)
                             : bpk::launch_sparse(a, kupd, G->stream);
        if (e != hipSuccess) return hip_fail(e, dense ? "dense update launch" : "sparse update launch");
        if (schedule == BP_SCHED_SYNC) G->cur ^= 1;
        else G->cb_pass++;
    }
    return BP_OK;
}

}  // namespace bpi

size_t bp_align_up(size_t v, size_t a) { return bpi::align_up(v, a); }

namespace bpi {
namespace {
struct Roctx {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
};
const Roctx& roctx() {
    static const Roctx r = [] {
        Roctx x;
        const char* e = std::getenv("BP_ROCTX");
        if (!e || std::strcmp(e, "1") != 0) return x;
        // the rocprofiler-sdk roctx (what rocprofv3 records), then the older one
        void* h = nullptr;
        for (const char* lib : {"librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1",
                                "libroctx64.so", "/opt/rocm/lib/libroctx64.so"})
            if (!h) h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
        if (!h) return x;
        x.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
        x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        if (!x.push || !x.pop) x = Roctx{};
        return x;
    }();
    return r;
}
}  // namespace

TraceRange::TraceRange(const char* name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name);
}
TraceRange::~TraceRange() {
    if (on) roctx().pop();
}
}  // namespace bpi

using namespace bpi;

extern "C" {

int bp_set_sync_fusion(bp_grid* G, int32_t enable) {
    if (!G) return fail(BP_EINVAL, "null handle");
    G->fuse_sync = enable != 0;
    return BP_OK;
}

int bp_message_stats(bp_grid* G, float* max_change, int32_t* non_finite) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!max_change && !non_finite) return fail(BP_EINVAL, "no output");
    if (!G->pot_set || !G->ws) return fail(BP_ESTATE, "no potential or no workspace");
    int st = with_device(G);
    if (st) return st;
    hipError_t e = bpk::launch_message_stats(G->msg[G->cur], G->msg[G->cur ^ 1], (size_t)4 * G->N * G->M,
                                             max_change, non_finite, G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "message stats launch");
}

static_assert(BP_PAIR_STRIPS == bpk::kPairStrips && BP_PAIR_BANDS == bpk::kPairBands &&
                  BP_PAIR_SLOTS == bpk::kPairSlots && BP_PAIR_WIDE == bpk::kPairWide &&
                  BP_PAIR_WALK == bpk::kPairWalk && BP_PAIR_TILE == bpk::kPairTile,
              "the header's layouts are the kernels'");

int bp_set_launch_tuning(bp_grid* G, int32_t layout, int32_t cap) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (layout < BP_PAIR_STRIPS || layout > BP_PAIR_TILE) return fail(BP_EINVAL, "bad layout %d", layout);
    if (cap < -1 || cap > 64) return fail(BP_EINVAL, "bad workgroups-per-CU cap %d", cap);
    G->pair_layout = layout;
    G->pair_cap = cap;
    G->pair_layout_set = true;
    return BP_OK;
}

int bp_get_launch_tuning(const bp_grid* G, int32_t* layout, int32_t* cap) {
    if (!G || !layout || !cap) return fail(BP_EINVAL, "null argument");
    *layout = G->pair_layout;
    *cap = G->pair_cap;
    return BP_OK;
}

int bp_autotune(bp_grid* G, int32_t mode, int32_t schedule, int32_t trial_iters, float* best_us) {
    TraceRange tr("bp_autotune");
    int st = check_ready(G);
    if (st) return st;
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (schedule != BP_SCHED_SYNC && schedule != BP_SCHED_CHECKERBOARD)
        return fail(BP_EINVAL, "autotune covers the synchronous and checkerboard schedules");
    if (trial_iters < 2 || trial_iters % 2) return fail(BP_EINVAL, "trial_iters must be even and >= 2");
    if ((st = with_device(G))) return st;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    // The current setting is timed first; another replaces the best only when
    // at least 1% faster, so that timing noise does not flip between
    // near-equal mappings from run to run.
    const int layout0 = G->pair_layout, cap0 = G->pair_cap;
    float best = 1e30f;
    int best_layout = layout0, best_cap = cap0;
    struct Cand { int layout, cap; };
    std::vector<Cand> cands = {{layout0, cap0}};
    for (int layout : {BP_PAIR_WIDE, BP_PAIR_STRIPS, BP_PAIR_BANDS, BP_PAIR_SLOTS})
        for (int cap : {0, 4, 3}) cands.push_back({layout, cap});
    cands.push_back({BP_PAIR_WALK, -1});
    cands.push_back({BP_PAIR_TILE, -1});
    // Two rounds over the candidates, each candidate keeping its faster
    // trial: the clock drifts while the trials run, and a single pass lets
    // that drift, rather than the mapping, decide between near-equal ones.
    std::vector<float> trial(cands.size(), 1e30f);
    for (int round = 0; round < 2 && !st; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Cand& c = cands[ci];
            G->pair_layout = c.layout;
            G->pair_cap = c.cap;
            if ((st = iterate(G, mode, 2, schedule, false))) break;  // warm
            e = hipEventRecord(e0, G->stream);
            if (e == hipSuccess && (st = iterate(G, mode, trial_iters, schedule, false))) break;
            if (e == hipSuccess) e = hipEventRecord(e1, G->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = hip_fail(e, "autotune trial");
                break;
            }
            trial[ci] = std::min(trial[ci], ms);
        }
    }
    for (size_t ci = 0; ci < cands.size() && !st; ++ci) {
        if (trial[ci] < 0.99f * best) {
            best = trial[ci];
            best_layout = cands[ci].layout;
            best_cap = cands[ci].cap;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    G->pair_layout = st ? layout0 : best_layout;
    G->pair_cap = st ? cap0 : best_cap;
    if (!st) G->pair_layout_set = true;
    if (st) return st;
    if (best_us) *best_us = best * 1000.0f / trial_iters;
    return bp_reset_messages(G);
}

int bp_set_arithmetic(bp_grid* G, int32_t arith) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (arith != BP_ARITH_F64 && arith != BP_ARITH_F32) return fail(BP_EINVAL, "bad arithmetic %d", arith);
    G->arith_f32 = arith == BP_ARITH_F32;
    // the default mapping follows the arithmetic: the tile launch for float32
    // (where it applies; elsewhere it runs the wide strips), wide strips for double
    if (!G->pair_layout_set) G->pair_layout = G->arith_f32 ? bpk::kPairTile : bpk::kPairWide;
    return BP_OK;
}

int bp_init_grid(bp_grid** out, int32_t H, int32_t W, void* hip_stream) {
    if (!out) return fail(BP_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (H < 1 || W < 1) return fail(BP_EINVAL, "grid %d x %d: both sides must be >= 1", H, W);
    if ((int64_t)H * W >= (int64_t(1) << 29)) return fail(BP_EINVAL, "grid too large");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int count = 0;
    e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(BP_EHIP, "no HIP device available");
    bp_grid* G = new (std::nothrow) bp_grid();
    if (!G) return fail(BP_ENOMEM, "host allocation failed");
    G->dev = dev;
    G->stream = static_cast<hipStream_t>(hip_stream);
    G->H = H;
    G->W = W;
    G->N = H * W;
    *out = G;
    return BP_OK;
}

int bp_set_stream(bp_grid* G, void* hip_stream) {
    if (!G) return fail(BP_EINVAL, "null handle");
    G->stream = static_cast<hipStream_t>(hip_stream);
    return BP_OK;
}

int bp_set_potential(bp_grid* G, int32_t M, int32_t T, float alpha, float fbar) {
    if (!G) return fail(BP_EINVAL, "null handle");
    invalidate_grad(G);
    if (M < 1 || M > BP_MAX_LABELS) return fail(BP_EINVAL, "M=%d outside [1, %d]", M, BP_MAX_LABELS);
    if (T < 0 || T >= M) return fail(BP_EINVAL, "T=%d outside [0, M-1]", T);
    if (!std::isfinite(alpha)) return fail(BP_EINVAL, "alpha not finite");
    const bool tied = fbar == BP_FBAR_TIED;
    if (tied) fbar = (float)std::exp(-(double)alpha * T);
    if (!std::isfinite(fbar) || fbar < 0.0f)
        return fail(BP_EINVAL, "fbar must be finite and >= 0 (or BP_FBAR_TIED)");
    if (M != G->M) {
        G->ws = nullptr;
        G->ws_bytes = 0;
        G->msg[0] = G->msg[1] = nullptr;
        G->g = nullptr;
    }
    G->M = M;
    G->T = T;
    G->alpha = alpha;
    G->fbar = fbar;
    G->fbar_tied = tied;
    build_tables(G);
    G->pot_set = true;
    G->general = false;        // back to the window potential
    G->win_tab_valid = false;  // its Eq. 10 tables follow T, alpha and fbar
    return BP_OK;
}

int64_t bp_workspace_bytes(const bp_grid* G) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    return (int64_t)(validate_flag_offset(G) + 256);
}

int bp_attach_workspace(bp_grid* G, void* dev_ptr, int64_t bytes) {
    if (!G) return fail(BP_EINVAL, "null handle");
    invalidate_grad(G);
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    if (!dev_ptr) return fail(BP_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(BP_EINVAL, "workspace not 256-byte aligned");
    const int64_t need = bp_workspace_bytes(G);
    if (bytes < need) return fail(BP_ENOMEM, "workspace %lld bytes < %lld needed", (long long)bytes, (long long)need);
    G->ws = dev_ptr;
    G->ws_bytes = bytes;
    const size_t buf = align_up(G->msg_floats() * sizeof(float), 256);
    BP_ASSERT(2 * buf <= validate_flag_offset(G));
    BP_ASSERT(validate_flag_offset(G) + 256 <= (size_t)bytes);
    G->msg[0] = static_cast<float*>(dev_ptr);
    G->msg[1] = reinterpret_cast<float*>(static_cast<char*>(dev_ptr) + buf);
    return bp_reset_messages(G);
}

int bp_set_unary(bp_grid* G, const float* g_dev) {
    if (!G) return fail(BP_EINVAL, "null handle");
    invalidate_grad(G);
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    if (!g_dev) return fail(BP_EINVAL, "null unary");
    if (reinterpret_cast<uintptr_t>(g_dev) % 16) return fail(BP_EINVAL, "unary not 16-byte aligned");
    const char* v = std::getenv("BP_VALIDATE");
    if (v && v[0] == '1') {
        // A row with a negative or non-finite entry, or with no positive
        // entry, would make every message from that pixel 0/0 (Eq. 5 and the
        // normalisation): check on the device and wait for the answer.
        if (!G->ws) return fail(BP_ESTATE, "BP_VALIDATE checks need the workspace attached first");
        int st = with_device(G);
        if (st) return st;
        int* flag = reinterpret_cast<int*>(static_cast<char*>(G->ws) + validate_flag_offset(G));
        hipError_t e = bpk::launch_validate_unary(g_dev, G->N, G->M, flag, G->stream);
        int bad = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, G->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(G->stream);
        if (e != hipSuccess) return hip_fail(e, "unary validation");
        if (bad)
            return fail(BP_EINVAL, "unary has a negative or non-finite entry, or a row with no positive entry");
    }
    G->g = g_dev;
    return BP_OK;
}

int bp_reset_messages(bp_grid* G) {
    if (!G) return fail(BP_EINVAL, "null handle");
    invalidate_grad(G);
    if (!G->ws) return fail(BP_ESTATE, "no workspace attached");
    int st = with_device(G);
    if (st) return st;
    G->cur = 0;
    G->cb_pass = 0;
    // The current buffer in full; in the other, the slots no update writes
    // (those of off-grid neighbours), so that they read 1/M whichever buffer
    // is current: the first launch into it writes every other slot.
    hipError_t e = bpk::launch_fill(G->msg[0], G->msg_floats(), 1.0f / (float)G->M, G->stream);
    if (e != hipSuccess) return hip_fail(e, "message reset");
    e = bpk::launch_fill_border(G->msg[1], G->H, G->W, G->M, 1.0f / (float)G->M, G->stream);
    if (e != hipSuccess) return hip_fail(e, "message reset");
    return BP_OK;
}

int bp_iterate(bp_grid* G, int32_t mode, int32_t n_iters, int32_t schedule) {
    TraceRange tr("bp_iterate");
    return iterate(G, mode, n_iters, schedule, false);
}

int bp_iterate_dense(bp_grid* G, int32_t mode, int32_t n_iters, int32_t schedule) {
    TraceRange tr("bp_iterate_dense");
    return iterate(G, mode, n_iters, schedule, true);
}

static int readout(bp_grid* G, float* beliefs, int32_t* labels) {
    TraceRange tr("bp_readout");
    int st = check_ready(G);
    if (st) return st;
    if ((st = with_device(G))) return st;
    UpdateArgs a = base_args(G, G->msg[G->cur], nullptr, -1);
    hipError_t e = bpk::launch_readout(a, beliefs, labels, G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "readout launch");
}

int bp_beliefs(bp_grid* G, float* out_dev) {
    if (!out_dev) return fail(BP_EINVAL, "null beliefs output");
    if (reinterpret_cast<uintptr_t>(out_dev) % 16) return fail(BP_EINVAL, "beliefs output not 16-byte aligned");
    return readout(G, out_dev, nullptr);
}

int bp_map_labels(bp_grid* G, int32_t* out_dev) {
    if (!out_dev) return fail(BP_EINVAL, "null labels output");
    return readout(G, nullptr, out_dev);
}

int bp_readout(bp_grid* G, float* beliefs_dev, int32_t* labels_dev) {
    if (!beliefs_dev && !labels_dev) return fail(BP_EINVAL, "null beliefs and labels outputs");
    if (reinterpret_cast<uintptr_t>(beliefs_dev) % 16) return fail(BP_EINVAL, "beliefs output not 16-byte aligned");
    return readout(G, beliefs_dev, labels_dev);
}

int bp_get_messages(const bp_grid* G, float* dst_dev) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->ws) return fail(BP_ESTATE, "no workspace attached");
    if (!dst_dev) return fail(BP_EINVAL, "null destination");
    int st = with_device(G);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(dst_dev, G->msg[G->cur], G->msg_floats() * sizeof(float),
                                  hipMemcpyDeviceToDevice, G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipMemcpyAsync (get messages)");
}

int bp_set_messages(bp_grid* G, const float* src_dev) {
    if (!G) return fail(BP_EINVAL, "null handle");
    invalidate_grad(G);
    if (!G->ws) return fail(BP_ESTATE, "no workspace attached");
    if (!src_dev) return fail(BP_EINVAL, "null source");
    if (reinterpret_cast<uintptr_t>(src_dev) % 16) return fail(BP_EINVAL, "source not 16-byte aligned");
    int st = with_device(G);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(G->msg[G->cur], src_dev, G->msg_floats() * sizeof(float),
                                  hipMemcpyDeviceToDevice, G->stream);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipMemcpyAsync (set messages)");
}

int bp_destroy(bp_grid* G) {
    delete G;
    return BP_OK;
}

const char* bp_status_string(int status) {
    switch (status) {
        case BP_OK: return "BP_OK";
        case BP_EINVAL: return "BP_EINVAL: invalid argument";
        case BP_ESTATE: return "BP_ESTATE: call out of order";
        case BP_ENOMEM: return "BP_ENOMEM: workspace too small or allocation failed";
        case BP_EHIP: return "BP_EHIP: HIP runtime error";
        case BP_EUNSUPPORTED: return "BP_EUNSUPPORTED: not supported";
        default: return "unknown status";
    }
}

const char* bp_last_error(void) { return g_last_error; }

}  // extern "C"
