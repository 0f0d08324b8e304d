// Host driver of the adjoint: checkpointed forward and segment-wise reverse
// pass over unrolled synchronous sum-product BP.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/bp.h"
#include "bp_adjoint.hpp"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using namespace bpi;

namespace {

// Workspace plan for n iterations with a checkpoint every k.
struct GradLayout {
    int n, k, nseg, nckpt;
    size_t buf;        // bytes of one message state (aligned)
    size_t ckpt_off, seg_off, lam_off, part_off, total;
    unsigned blocks;   // workgroups of one adjoint launch = partial slots

    GradLayout(const bp_grid* G, int n_, int k_) : n(n_), k(k_) {
        nseg = n > 0 ? (n + k - 1) / k : 0;
        nckpt = nseg > 1 ? nseg - 1 : 0;
        buf = bp_align_up(G->msg_floats() * sizeof(float), 256);
        blocks = bpk::adjoint_blocks(G->M, G->N);
        ckpt_off = 0;
        seg_off = ckpt_off + (size_t)nckpt * buf;
        lam_off = seg_off + (size_t)(n > 0 ? (k < n ? k : n) : 0) * buf;
        part_off = lam_off + 2 * buf;
        total = part_off + bp_align_up(blocks * sizeof(float), 256);
        BP_ASSERT(ckpt_off <= seg_off && seg_off <= lam_off && lam_off + 2 * buf == part_off && part_off < total);
        BP_ASSERT(seg_off == (size_t)nckpt * buf && nckpt <= nseg);
    }
    float* ckpt(char* ws, int i) const { return reinterpret_cast<float*>(ws + ckpt_off + i * buf); }
    float* seg(char* ws, int i) const { return reinterpret_cast<float*>(ws + seg_off + i * buf); }
    float* lam(char* ws, int i) const { return reinterpret_cast<float*>(ws + lam_off + i * buf); }
    float* part(char* ws) const { return reinterpret_cast<float*>(ws + part_off); }
};

int grad_checks(const bp_grid* G, int n, int k) {
    int st = check_ready(G);
    if (st) return st;
    if (n < 0) return fail(BP_EINVAL, "n_iters < 0");
    if (k < 1) return fail(BP_EINVAL, "ckpt_every must be >= 1");
    if (G->general) return fail(BP_EUNSUPPORTED, "the adjoint takes the truncated-linear potential only");
    // The reverse pass works with log-message adjoints and divides by u(y);
    // fbar > 0 keeps every u(y) >= fbar * sum(h) > 0.  With fbar = 0, u(y) is
    // 0 wherever h vanishes across the window, and the log adjoint carries
    // no information there.
    if (!(G->fbar_d > 0.0)) return fail(BP_EUNSUPPORTED, "the adjoint needs fbar > 0 (messages stay positive)");
    if (!bpk::adjoint_supported(G->M, G->T))
        return fail(BP_EUNSUPPORTED, "adjoint supports T <= 16 (12 for M <= 16) (M=%d, T=%d)", G->M, G->T);
    return BP_OK;
}

// One synchronous sum-product iteration in -> out, or two (pair) with the
// intermediate state into mid (null: not kept).
hipError_t sync_sum_step(bp_grid* G, const float* in, float* out, bool pair = false, float* mid = nullptr) {
    bpk::UpdateArgs a = base_args(G, in, out, -1);
    memcpy(a.tab, G->tab_w, sizeof a.tab);
    a.mid = mid;
    return pair ? bpk::launch_sparse2(a, bpk::kSum, G->stream) : bpk::launch_sparse(a, bpk::kSum, G->stream);
}

}  // namespace

extern "C" {

int64_t bp_grad_workspace_bytes(const bp_grid* G, int32_t n_iters, int32_t ckpt_every) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    if (n_iters < 0 || ckpt_every < 1) return fail(BP_EINVAL, "n_iters >= 0 and ckpt_every >= 1 required");
    return (int64_t)GradLayout(G, n_iters, ckpt_every).total;
}

int bp_forward_ckpt(bp_grid* G, int32_t n_iters, int32_t ckpt_every, void* gws, int64_t bytes) {
    bpi::TraceRange tr("bp_forward_ckpt");
    int st = grad_checks(G, n_iters, ckpt_every);
    if (st) return st;
    if (!gws) return fail(BP_EINVAL, "null gradient workspace");
    if (reinterpret_cast<uintptr_t>(gws) % 256) return fail(BP_EINVAL, "gradient workspace not 256-byte aligned");
    const GradLayout L(G, n_iters, ckpt_every);
    if (bytes < (int64_t)L.total)
        return fail(BP_ENOMEM, "gradient workspace %lld bytes < %zu needed", (long long)bytes, L.total);
    if ((st = bp_reset_messages(G))) return st;  // also clears any previous gradient state
    char* ws = static_cast<char*>(gws);
    // Route outputs: the state after iteration j*k goes straight into
    // checkpoint j-1, every other kept state into a ping-pong buffer, so the
    // checkpoints cost no copies.  Between checkpoints no state is kept, so
    // iterations run two per launch where the pair kernel is compiled (the
    // same bits as single launches).
    const bool pairs = G->fuse_sync && bpk::sparse2_supported(G->M, G->T);
    float* src = G->msg[0];
    for (int t = 0; t < n_iters;) {
        const int boundary = std::min(n_iters, (t / ckpt_every + 1) * ckpt_every);  // next kept state
        const int step = (pairs && boundary - t >= 2) ? 2 : 1;
        const int done = t + step;
        float* dst;
        if (done % ckpt_every == 0 && done < n_iters) dst = L.ckpt(ws, done / ckpt_every - 1);
        else dst = (src == G->msg[0]) ? G->msg[1] : G->msg[0];
        hipError_t e = sync_sum_step(G, src, dst, step == 2);
        if (e != hipSuccess) return hip_fail(e, "forward update launch");
        src = dst;
        t = done;
    }
    G->cur = (src == G->msg[0]) ? 0 : 1;
    G->grad_ready = true;
    G->grad_n = n_iters;
    G->grad_k = ckpt_every;
    G->grad_ws = ws;
    return BP_OK;
}

int bp_backward(bp_grid* G, const float* dL_db, float* dtheta, float* dalpha) {
    bpi::TraceRange tr("bp_backward");
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->grad_ready) return fail(BP_ESTATE, "bp_backward needs a bp_forward_ckpt with no state change since");
    if (!dL_db || !dtheta || !dalpha) return fail(BP_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(dL_db) % 16 || reinterpret_cast<uintptr_t>(dtheta) % 16)
        return fail(BP_EINVAL, "dL_db and dtheta must be 16-byte aligned");
    int st = with_device(G);
    if (st) return st;
    const int n = G->grad_n, k = G->grad_k;
    const GradLayout L(G, n, k);
    char* ws = G->grad_ws;
    hipStream_t s = G->stream;
    hipError_t e = bpk::launch_fill(L.part(ws), L.blocks, 0.0f, s);
    if (e != hipSuccess) return hip_fail(e, "partials reset");

    bpk::SeedArgs sa;
    sa.g = G->g;
    sa.m = G->msg[G->cur];
    sa.dL_db = dL_db;
    sa.theta_bar = dtheta;
    sa.lam_out = L.lam(ws, 0);
    sa.H = G->H; sa.W = G->W; sa.M = G->M; sa.N = G->N;
    if ((e = bpk::launch_adjoint_seed(sa, s)) != hipSuccess) return hip_fail(e, "adjoint seed launch");

    bpk::AdjointArgs aa;
    memset(&aa, 0, sizeof aa);
    aa.g = G->g;
    aa.theta_bar = dtheta;
    aa.alpha_part = L.part(ws);
    aa.H = G->H; aa.W = G->W; aa.M = G->M; aa.N = G->N;
    aa.fbar = G->fbar;
    aa.fbar_d = G->fbar_d;
    const double dfbar = G->fbar_tied ? -(double)G->T * std::exp(-(double)G->alpha * G->T) : 0.0;
    aa.dfbar = (float)dfbar;
    for (int d = 0; d < bpk::kAdjTab; ++d) {
        const bool in = d <= G->T;
        const double f = std::exp(-(double)G->alpha * d);
        aa.w[d] = in ? G->tab_w[d] : 0.0f;
        aa.wd[d] = in ? f - G->fbar_d : 0.0;
        aa.dw[d] = in ? (float)(-(double)d * f - dfbar) : 0.0f;
    }
    int lcur = 0;
    for (int sidx = L.nseg - 1; sidx >= 0; --sidx) {
        const int t0 = sidx * k;
        const int len = (n - t0) < k ? (n - t0) : k;
        // state m^{t0}: a checkpoint, or the uniform start
        const float* state0;
        if (sidx == 0) {
            if ((e = bpk::launch_fill(L.seg(ws, 0), G->msg_floats(), 1.0f / (float)G->M, s)) != hipSuccess)
                return hip_fail(e, "uniform start");
            state0 = L.seg(ws, 0);
        } else {
            state0 = L.ckpt(ws, sidx - 1);
        }
        // recompute m^{t0+1} .. m^{t0+len-1} into seg[1 .. len-1], two per
        // launch where the pair kernel is compiled (it stores the first of the
        // two states too)
        const bool pairs = G->fuse_sync && bpk::sparse2_supported(G->M, G->T);
        const float* prev = state0;
        for (int i = 1; i < len;) {
            const bool two = pairs && i + 1 < len;
            if ((e = sync_sum_step(G, prev, L.seg(ws, two ? i + 1 : i), two, two ? L.seg(ws, i) : nullptr)) !=
                hipSuccess)
                return hip_fail(e, "recompute launch");
            prev = L.seg(ws, two ? i + 1 : i);
            i += two ? 2 : 1;
        }
        for (int i = len - 1; i >= 0; --i) {
            const int t = t0 + i;
            aa.m = i == 0 ? state0 : L.seg(ws, i);
            aa.lam_in = L.lam(ws, lcur);
            aa.lam_out = t > 0 ? L.lam(ws, lcur ^ 1) : nullptr;
            if ((e = bpk::launch_adjoint_step(aa, G->T, s)) != hipSuccess) return hip_fail(e, "adjoint step launch");
            lcur ^= 1;
        }
    }
    if ((e = bpk::launch_sum_partials(L.part(ws), (int)L.blocks, dalpha, s)) != hipSuccess)
        return hip_fail(e, "alpha reduction launch");
    return BP_OK;
}

}  // extern "C"
