// Coarse-to-fine (multi-scale) BP in tandem with the O(mM) update (Sec. 2,
// Sec. 6): a pyramid of 2 x 2 block unaries, the coarsest level solved from
// uniform messages, every finer level started from its parent's inbox.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/bp.h"
#include "bp_internal.hpp"
#include "bp_kernels.hpp"
#include "bp_launch.hpp"

using namespace bpi;

namespace bpk {
namespace {

// Unary of block (r, c) at the next level: the product of its (up to four)
// children in double, divided by its maximum over labels, rounded once.
template <int G>
__global__ __launch_bounds__(kBlock) void pyramid_kernel(const float* __restrict__ fine, int Hf, int Wf,
                                                         float* __restrict__ coarse, int Hc, int Wc, int M) {
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    if (slot >= Hc * Wc) return;  // whole groups
    const int r = slot / Wc, c = slot - (slot / Wc) * Wc;
    const int x0 = pos * kLpl;
    const bool full = M == G * kLpl;
    double p[kLpl] = {1.0, 1.0, 1.0, 1.0};
#pragma unroll
    for (int dr = 0; dr < 2; ++dr)
#pragma unroll
        for (int dc = 0; dc < 2; ++dc) {
            const int fr = 2 * r + dr, fc = 2 * c + dc;
            if (fr < Hf && fc < Wf) {
                float v[kLpl];
                load_labels<false>(fine + ((size_t)fr * Wf + fc) * M, x0, M, full, v, 0.0f);
#pragma unroll
                for (int i = 0; i < kLpl; ++i) p[i] *= v[i];
            }
        }
    const double mx = group_max_d<G>(fmax(fmax(p[0], p[1]), fmax(p[2], p[3])));
    float out[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) out[i] = (float)(p[i] / mx);
    store_labels<false>(coarse + (size_t)slot * M, x0, M, full, out);
}

// Initial inbox of a level: pixel (r, c) copies the inbox of block
// (r/2, c/2), into fine0 in full and into fine1 either in full (all1) or
// only in the slots of off-grid neighbours, the ones no update writes.
// blockIdx.y walks the (slot k, row r) rows of the [4][Hf][Wf][M] buffers; a
// thread moves VEC consecutive labels of one pixel (VEC = 4: M is a multiple
// of 4, so rows stay 16-byte aligned).
template <int VEC>
__global__ __launch_bounds__(kBlock) void prolong_kernel(const float* __restrict__ coarse, int Hc, int Wc,
                                                         float* __restrict__ fine0, float* __restrict__ fine1,
                                                         int all1, int Hf, int Wf, int M) {
    typedef float vec_t __attribute__((ext_vector_type(VEC)));
    const int mv = M / VEC;   // vectors per pixel
    const int row_v = Wf * mv;  // vectors per fine row
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= row_v) return;
    const int c = j / mv, xv = j - c * mv;
    for (int kr = blockIdx.y; kr < 4 * Hf; kr += gridDim.y) {
        const int k = kr / Hf, r = kr - k * Hf;
        const size_t src = (((size_t)k * Hc + r / 2) * Wc + c / 2) * mv + xv;
        const size_t dst = (size_t)kr * row_v + j;
        const vec_t v = reinterpret_cast<const vec_t*>(coarse)[src];
        reinterpret_cast<vec_t*>(fine0)[dst] = v;
        const bool off_grid = (k == kLeft && c == 0) || (k == kRight && c == Wf - 1) || (k == kUp && r == 0) ||
                              (k == kDown && r == Hf - 1);
        if (all1 || off_grid) reinterpret_cast<vec_t*>(fine1)[dst] = v;
    }
}

template <int G>
hipError_t go_pyramid(const float* fine, int Hf, int Wf, float* coarse, int Hc, int Wc, int M, hipStream_t s) {
    const unsigned blocks = (unsigned)(((size_t)Hc * Wc + (kBlock / G) - 1) / (kBlock / G));
    hipLaunchKernelGGL((pyramid_kernel<G>), dim3(blocks), dim3(kBlock), 0, s, fine, Hf, Wf, coarse, Hc, Wc, M);
    return hipGetLastError();
}

hipError_t launch_pyramid(const float* fine, int Hf, int Wf, float* coarse, int Hc, int Wc, int M, hipStream_t s) {
    switch (lanes_for(M)) {
        case 4: return go_pyramid<4>(fine, Hf, Wf, coarse, Hc, Wc, M, s);
        case 8: return go_pyramid<8>(fine, Hf, Wf, coarse, Hc, Wc, M, s);
        case 16: return go_pyramid<16>(fine, Hf, Wf, coarse, Hc, Wc, M, s);
        case 32: return go_pyramid<32>(fine, Hf, Wf, coarse, Hc, Wc, M, s);
        default: return go_pyramid<64>(fine, Hf, Wf, coarse, Hc, Wc, M, s);
    }
}

hipError_t launch_prolong(const float* coarse, int Hc, int Wc, float* fine0, float* fine1, bool all1, int Hf,
                          int Wf, int M, hipStream_t s) {
    const int vec = M % 4 == 0 ? 4 : 1;
    const unsigned bx = (unsigned)(((size_t)Wf * (M / vec) + kBlock - 1) / kBlock);
    const dim3 grid(bx, (unsigned)std::min(4 * Hf, 65535));
    if (vec == 4)
        hipLaunchKernelGGL(prolong_kernel<4>, grid, dim3(kBlock), 0, s, coarse, Hc, Wc, fine0, fine1, (int)all1, Hf, Wf,
                           M);
    else
        hipLaunchKernelGGL(prolong_kernel<1>, grid, dim3(kBlock), 0, s, coarse, Hc, Wc, fine0, fine1, (int)all1, Hf, Wf,
                           M);
    return hipGetLastError();
}

}  // namespace
}  // namespace bpk

namespace {

constexpr int kMaxLevels = 12;

struct Level {
    int H, W;
    size_t unary_off, msg_off[2];  // byte offsets in the multi-scale workspace (levels >= 1)
};

std::vector<Level> plan_levels(const bp_grid* G, int levels, size_t* total) {
    std::vector<Level> L(levels + 1);
    L[0].H = G->H;
    L[0].W = G->W;
    size_t off = 0;
    for (int l = 1; l <= levels; ++l) {
        L[l].H = (L[l - 1].H + 1) / 2;
        L[l].W = (L[l - 1].W + 1) / 2;
        const size_t n = (size_t)L[l].H * L[l].W * G->M;
        L[l].unary_off = off;
        off += bp_align_up(n * sizeof(float), 256);
        for (int b = 0; b < 2; ++b) {
            L[l].msg_off[b] = off;
            off += bp_align_up(4 * n * sizeof(float), 256);
        }
    }
    *total = off;
    for (int l = 1; l <= levels; ++l) {
        BP_ASSERT(L[l].unary_off % 256 == 0 && L[l].msg_off[0] % 256 == 0 && L[l].msg_off[1] % 256 == 0);
        BP_ASSERT(L[l].unary_off < L[l].msg_off[0] && L[l].msg_off[0] < L[l].msg_off[1] && L[l].msg_off[1] < off);
        BP_ASSERT(L[l].H >= 1 && L[l].W >= 1 && 2 * L[l].H >= L[l - 1].H && 2 * L[l].W >= L[l - 1].W);
    }
    return L;
}

}  // namespace

extern "C" {

int64_t bp_multiscale_workspace_bytes(const bp_grid* G, int32_t levels) {
    if (!G) return fail(BP_EINVAL, "null handle");
    if (!G->pot_set) return fail(BP_ESTATE, "bp_set_potential has not been called");
    if (levels < 0 || levels > kMaxLevels) return fail(BP_EINVAL, "levels must be in [0, %d]", kMaxLevels);
    size_t total = 0;
    plan_levels(G, levels, &total);
    return (int64_t)std::max<size_t>(total, 256);
}

int bp_iterate_multiscale(bp_grid* G, int32_t mode, int32_t levels, const int32_t* iters, void* ms_ws,
                          int64_t ms_bytes) {
    TraceRange tr("bp_iterate_multiscale");
    int st = check_ready(G);
    if (st) return st;
    invalidate_grad(G);
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (levels < 0 || levels > kMaxLevels) return fail(BP_EINVAL, "levels must be in [0, %d]", kMaxLevels);
    if (!iters) return fail(BP_EINVAL, "null iteration counts");
    for (int l = 0; l <= levels; ++l)
        if (iters[l] < 0) return fail(BP_EINVAL, "iters[%d] < 0", l);
    // Edge type maps describe the finest grid only; one potential shared by
    // every edge is the same at every level.
    if (G->general && (G->type_h || G->type_v))
        return fail(BP_EUNSUPPORTED, "multi-scale BP takes one potential for every edge (no type maps)");
    // Max-product of the window potential with fbar above some f(d) needs
    // Eq. 10: the window kernel's Eq. 10 form, or the general kernel over
    // the window's tables beyond the register windows (as bp_iterate).
    const bool eq10 = !G->general && mode == BP_MAX_PRODUCT && !max_product_ok(G);
    const bool eq10_general = eq10 && bpk::sparse_variant_tw(G->M, G->T) < 0;
    const bool general = G->general || eq10_general;
    size_t need = 0;
    std::vector<Level> L = plan_levels(G, levels, &need);
    if (levels > 0) {
        if (!ms_ws || reinterpret_cast<uintptr_t>(ms_ws) % 256)
            return fail(BP_EINVAL, "multi-scale workspace null or not 256-byte aligned");
        if (ms_bytes < (int64_t)need)
            return fail(BP_ENOMEM, "multi-scale workspace %lld bytes < %zu needed", (long long)ms_bytes, need);
    }
    if ((st = with_device(G))) return st;
    if (eq10_general && (st = build_window_tables(G))) return st;
    const int kmode = mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax;
    char* base = static_cast<char*>(ms_ws);
    auto unary = [&](int l) { return l == 0 ? G->g : reinterpret_cast<const float*>(base + L[l].unary_off); };
    auto buf = [&](int l, int b) {
        return l == 0 ? G->msg[b] : reinterpret_cast<float*>(base + L[l].msg_off[b]);
    };
    hipError_t e;
    for (int l = 1; l <= levels; ++l) {
        e = bpk::launch_pyramid(unary(l - 1), L[l - 1].H, L[l - 1].W, const_cast<float*>(unary(l)), L[l].H, L[l].W,
                                G->M, G->stream);
        if (e != hipSuccess) return hip_fail(e, "pyramid launch");
    }
    int cur = 0;
    for (int l = levels; l >= 0; --l) {
        const size_t n = (size_t)4 * L[l].H * L[l].W * G->M;
        if (l == levels) {
            for (int b = 0; b < 2; ++b) {
                e = bpk::launch_fill(buf(l, b), n, 1.0f / (float)G->M, G->stream);
                if (e != hipSuccess) return hip_fail(e, "multi-scale reset");
            }
            cur = 0;
        } else {
            // Both buffers: slots of off-grid neighbours are never updated, and
            // a child's inbox copies its block's, off-grid slots included, so
            // they must hold the prolonged values whichever buffer is current.
            // The level's first update writes every other slot of buffer 1,
            // so with iterations to come only the off-grid ones are copied.
            e = bpk::launch_prolong(buf(l + 1, cur), L[l + 1].H, L[l + 1].W, buf(l, 0), buf(l, 1), iters[l] == 0,
                                    L[l].H, L[l].W, G->M, G->stream);
            if (e != hipSuccess) return hip_fail(e, "prolongation launch");
            cur = 0;
        }
        // synchronous iterations of this level, two per launch where the
        // window potential has a compiled pair kernel (same bits as singles)
        const bool pairs = !general && !eq10 && G->fuse_sync && bpk::sparse2_supported(G->M, G->T);
        for (int t = 0; t < iters[l];) {
            bpk::UpdateArgs a = base_args(G, buf(l, cur), buf(l, cur ^ 1), -1);
            a.g = unary(l);
            a.H = L[l].H;
            a.W = L[l].W;
            a.N = L[l].H * L[l].W;
            a.n_slots = a.N;
            a.half_w = (a.W + 1) / 2;
            if (general) {
                e = launch_general_update(G, a, kmode);
                t += 1;
            } else {
                memcpy(a.tab, kmode == bpk::kSum ? G->tab_w : G->tab_f, sizeof a.tab);
                a.eq10 = eq10;
                const bool two = pairs && iters[l] - t >= 2;
                e = two ? bpk::launch_sparse2(a, kmode, G->stream) : bpk::launch_sparse(a, kmode, G->stream);
                t += two ? 2 : 1;
            }
            if (e != hipSuccess) return hip_fail(e, "multi-scale update launch");
            cur ^= 1;
        }
    }
    G->cur = cur;
    G->cb_pass = 0;
    return BP_OK;
}

}  // extern "C"
