// Directional sweep schedule (Sec. 6): one sweep passes messages left, then
// right, then up, then down across the lattice.  A pass sends every message
// towards one direction, scanline by scanline (rows for left/right, columns
// for up/down), visiting the senders of a scanline from its far end so that
// each message uses the one its sender has just received from the opposite
// side.  Scanlines are independent; along one the updates are sequential.
//
// One group of G lanes walks one scanline.  The message a sender has just
// sent is exactly the inbox entry the next sender reads from the opposite
// side, so it stays in registers (the carry) as well as being stored for the
// later passes and the readout.  The unary and the two perpendicular inbox
// messages of a sender do not depend on the carry and are loaded eight steps
// ahead.  Those loads are unconditional, so that the ring of inputs in flight
// needs no copies and no branches: groups past the last scanline read the
// last one, the walk's tail re-reads its last sender, and a missing
// perpendicular neighbour reads the row of ones.  A pass writes only the
// inbox plane opposite to its direction and reads only the two perpendicular
// planes, so it runs in place, and the two passes of one axis run together in
// one launch.
#pragma once

#include <type_traits>

#include "bp_kernels.hpp"
#include "bp_walk.hpp"

namespace bpk {

constexpr int kSweepBlock = 64;  // one wave per workgroup: a pass has only H (or W) scanlines

// How a sender's message is computed: register window (the O(mM) update),
// LDS window with a runtime bound (wide T), the dense O(M^2) form, or the
// register window with Eq. 10 for max-product (max_message_eq10_d).
enum SweepKind { kSweepReg = 0, kSweepLds = 1, kSweepDense = 2, kSweepRegEq10 = 3 };

// LDS: the potential tables and each group's h (double).
constexpr size_t sweep_lds_bytes(int G, int M, int mode, int kind) {
    const size_t hbytes = (size_t)kSweepBlock * kLpl * sizeof(double);
    return kind == kSweepReg ? 0
         : kind == kSweepRegEq10 ? (size_t)(kSweepBlock / G) * eq10_row_doubles(G) * sizeof(double)
         : kind == kSweepLds ? kMaxTab * sizeof(double) + kMaxTab * sizeof(float) + hbytes
         : mode == kSum ? kMaxTab * sizeof(double) + (size_t)M * G * kLpl * sizeof(double) + hbytes
                        : (size_t)M * G * kLpl * sizeof(float) + hbytes;
}

// Direction and scanline block of this workgroup.  The two passes of one
// axis (left and right, or up and down) read only the two perpendicular
// inbox planes and write different planes, so one launch can run both:
// with a.both the second half of the grid runs opposite(a.dir).
__device__ __forceinline__ void sweep_block_dir(const UpdateArgs& a, int& blk, int& dir) {
    const int half = a.both ? (int)gridDim.x / 2 : (int)gridDim.x;
    const bool second = (int)blockIdx.x >= half;
    blk = second ? (int)blockIdx.x - half : (int)blockIdx.x;
    dir = second ? opposite(a.dir) : a.dir;
}

// The walk of one pass: group grp of the workgroup takes scanline
// blk * (kSweepBlock / G) + grp (sweep_block_dir).  msg(h, r, c, dir, m)
// turns the h of the sender at (r, c), sending towards dir, into its message
// m; it may hold block barriers, since every group of the workgroup makes
// the same number of steps (groups past the last scanline run on the last
// scanline's inputs and store nothing).  FULL: M == 4G.
template <int G, bool FULL, typename HT, typename Msg>
__device__ __forceinline__ void sweep_walk(const UpdateArgs& a, Msg&& msg) {
    constexpr int CAP = G * kLpl;
    constexpr int LPB = kSweepBlock / G;  // scanlines per workgroup
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    int blk, dir;
    sweep_block_dir(a, blk, dir);
    const bool horiz = dir == kLeft || dir == kRight;
    const bool forward = dir == kRight || dir == kDown;  // senders in increasing index
    const int n_lines = horiz ? a.H : a.W;
    const int len = horiz ? a.W : a.H;
    const bool live = blk * LPB + grp < n_lines;
    const int line = live ? blk * LPB + grp : n_lines - 1;  // the scanline whose inputs the group reads
    const int x0 = pos * kLpl;
    const size_t plane = (size_t)a.N * a.M;
    const int side0 = horiz ? kUp : kLeft;   // h = ((g * m_side0) * m_side1) * carry,
    const int side1 = horiz ? kDown : kRight;  // the product order of the other updates
    // the perpendicular inbox planes (up / left, down / right), or the row of
    // ones with a zero row stride where the scanline has no neighbour that side
    const float* in0 = line > 0 ? a.in + side0 * plane : kOnesRow.v;
    const float* in1 = line + 1 < n_lines ? a.in + side1 * plane : kOnesRow.v;
    const size_t stride0 = line > 0 ? (size_t)a.M : 0, stride1 = line + 1 < n_lines ? (size_t)a.M : 0;
    const int step_q = dir == kLeft ? -1 : dir == kRight ? 1 : dir == kUp ? -a.W : a.W;

    auto along = [&](int t) { return forward ? t : len - 1 - t; };  // position of the t-th sender
    auto sender = [&](int t) {  // pixel index of the t-th sender of this scanline
        const int s = along(t);
        return horiz ? line * a.W + s : s * a.W + line;
    };
    const int steps = len - 1;  // the last node of the scanline sends nothing this way
    if (steps <= 0) return;     // the same for every group
    // Consecutive senders are a fixed number of pixels apart, so the walk
    // advances pointers instead of recomputing offsets.
    const long dpix = (forward ? 1L : -1L) * (horiz ? 1L : (long)a.W);
    // inputs of the sender whose unary is at gp (and side rows at s0, s1)
    auto load_raw = [&](const float* gp, const float* s0, const float* s1, float (&gv)[kLpl], float (&m0)[kLpl],
                        float (&m1)[kLpl]) {
        load_labels<kUnaryNT>(gp, x0, a.M, FULL, gv, 0.0f);
        load_labels<kMsgNT>(s0, x0, a.M, FULL, m0, 1.0f);
        load_labels<kMsgNT>(s1, x0, a.M, FULL, m1, 1.0f);
    };

    // Inputs of the next kAhead senders in flight: a ring of registers,
    // statically indexed by unrolling the step loop by kAhead.  A step takes
    // about 0.4 us at one wave per SIMD, so eight steps cover a load's
    // latency; with twelve or more the ring no longer stays in registers.
    constexpr int kAhead = 8;
    float rg[kAhead][kLpl], r0[kAhead][kLpl], r1[kAhead][kLpl], carry[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) carry[i] = 1.0f;  // first sender: no carry
    // the next sender to load (t clamped to the last one) and its rows
    const long p0 = sender(0);
    const float* gp = a.g + p0 * a.M;
    const float* s0p = in0 + p0 * (long)stride0;
    const float* s1p = in1 + p0 * (long)stride1;
    const long dg = dpix * a.M, d0 = dpix * (long)stride0, d1 = dpix * (long)stride1;
    auto advance = [&](int t_loaded) {  // after loading sender t_loaded
        if (t_loaded + 1 < steps) {
            gp += dg;
            s0p += d0;
            s1p += d1;
        }
    };
#pragma unroll
    for (int j = 0; j < kAhead; ++j) {
        load_raw(gp, s0p, s1p, rg[j], r0[j], r1[j]);
        advance(j);
    }
    // where the t-th sender's message goes (receiver's inbox slot)
    float* op = a.out + opposite(dir) * plane + (p0 + step_q) * (long)a.M;
    for (int t0 = 0; t0 < steps; t0 += kAhead) {
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            const int t = t0 + j;
            if (t >= steps) break;  // the same for every group of the workgroup
            HT h[kLpl];  // Eq. 5, in the update's arithmetic (double, or float32 for kSumF32)
#pragma unroll
            for (int i = 0; i < kLpl; ++i) h[i] = (((HT)rg[j][i] * r0[j][i]) * r1[j][i]) * carry[i];
            load_raw(gp, s0p, s1p, rg[j], r0[j], r1[j]);
            advance(t + kAhead);
            float m[kLpl];
            const int s = along(t);
            msg(h, horiz ? line : s, horiz ? s : line, dir, m);
            if (live) store_labels<kMsgNT>(op, x0, a.M, FULL, m);
            op += dg;
#pragma unroll
            for (int i = 0; i < kLpl; ++i) carry[i] = m[i];
        }
    }
}

// sweep_walk for M = 4G and planes below 2^31 bytes, with the inputs
// staged through LDS instead of registers.  In the register ring the
// compiler cannot carry its load counts across the unrolled loop's back
// edge and waits for every load in flight once per kAhead steps, a full
// memory latency each time.  Here each step's three input rows (unary and
// the two perpendicular inbox rows; 16 bytes per lane, one 1 KB load per
// row for the wave) go by direct global-to-LDS loads into a ring of
// kStage slots, kStage steps ahead, and the waits are explicit: every step
// issues three loads and one buffer store (offset beyond the plane where
// the group has no scanline, and in the prologue), and memory operations
// complete in issue order, so a step's rows have landed once no more than
// the operations issued after them are outstanding.  The arithmetic and the
// order of the messages are sweep_walk's.
template <int G, typename HT, typename Msg>
__device__ __forceinline__ void sweep_walk_staged(const UpdateArgs& a, Msg&& msg) {
    static_assert(kSweepBlock == 64, "one wave per workgroup");
    constexpr int kStage = 16;
    __shared__ __attribute__((aligned(1024))) char ring[kStage][3][1024];
    constexpr int LPB = kSweepBlock / G;
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int lane = threadIdx.x & 63;
    int blk, dir;
    sweep_block_dir(a, blk, dir);
    const bool horiz = dir == kLeft || dir == kRight;
    const bool forward = dir == kRight || dir == kDown;
    const int n_lines = horiz ? a.H : a.W;
    const int len = horiz ? a.W : a.H;
    const bool live = blk * LPB + grp < n_lines;
    const int line = live ? blk * LPB + grp : n_lines - 1;
    const int M = 4 * G;
    const size_t plane = (size_t)a.N * M;
    const int side0 = horiz ? kUp : kLeft;
    const int side1 = horiz ? kDown : kRight;
    const float* in0 = line > 0 ? a.in + side0 * plane : kOnesRow.v;
    const float* in1 = line + 1 < n_lines ? a.in + side1 * plane : kOnesRow.v;
    const long stride0 = line > 0 ? M : 0, stride1 = line + 1 < n_lines ? M : 0;
    const int step_q = dir == kLeft ? -1 : dir == kRight ? 1 : dir == kUp ? -a.W : a.W;
    const int steps = len - 1;
    if (steps <= 0) return;  // the same for every group
    const long dpix = (forward ? 1L : -1L) * (horiz ? 1L : (long)a.W);
    const long p0 = horiz ? (long)line * a.W + (forward ? 0 : len - 1) : (long)(forward ? 0 : len - 1) * a.W + line;
    const int x0 = pos * kLpl;
    // this lane's 16 bytes of the t-th sender's rows (t clamped to the last)
    auto src = [&](int t, int k) -> const char* {
        const long p = p0 + (long)min(t, steps - 1) * dpix;
        const float* b = k == 0 ? a.g + p * M : k == 1 ? in0 + p * stride0 : in1 + p * stride1;
        return (const char*)(b + x0);
    };
    const uint32_t plane_b = (uint32_t)(plane * sizeof(float));
    const __amdgpu_buffer_rsrc_t out_r =
        __builtin_amdgcn_make_buffer_rsrc(a.out + opposite(dir) * plane, 0, (int)plane_b, kWalkRsrcWord3);
    const float zero[kLpl] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto issue = [&](int t) {
        char* dst = &ring[t % kStage][0][0];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            __builtin_amdgcn_global_load_lds((walk_gptr)src(t, k), (walk_lptr)(dst + k * 1024), 16, 0, 0);
    };
    // The compiler barriers keep each step's loads ahead of its store (a
    // store moved above a load would leave the wait one operation short).
#pragma unroll
    for (int t = 0; t < kStage; ++t) {
        issue(t);
        asm volatile("" ::: "memory");
        walk_store(out_r, kWalkDrop, zero);
        asm volatile("" ::: "memory");
    }
    float carry[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) carry[i] = 1.0f;  // first sender: no carry
    // The rows of step t + 1 are read from LDS during step t, off the
    // carried message's dependency chain.
    float rg[kLpl], r0[kLpl], r1[kLpl];
    auto read_rows = [&](int t) {
        const char* sl = &ring[t % kStage][0][0] + lane * 16;
        walk_read(sl, rg);
        walk_read(sl + 1024, r0);
        walk_read(sl + 2048, r1);
    };
    walk_wait<1 + 4 * (kStage - 1)>();  // step 0's loads
    asm volatile("" ::: "memory");
    read_rows(0);
    for (int t = 0; t < steps; ++t) {
        HT h[kLpl];  // Eq. 5, in the update's arithmetic, sweep_walk's factor order
#pragma unroll
        for (int i = 0; i < kLpl; ++i) h[i] = (((HT)rg[i] * r0[i]) * r1[i]) * carry[i];
        // step t + 1's loads: after them, the store of their step and four
        // operations for each of the kStage - 2 steps since
        walk_wait<1 + 4 * (kStage - 2)>();
        asm volatile("" ::: "memory");
        read_rows(t + 1);
        asm volatile("" ::: "memory");
        issue(t + kStage);  // into step t's slot, read before h above
        asm volatile("" ::: "memory");
        const long p = p0 + (long)t * dpix;
        const int s = horiz ? (int)(p - (long)line * a.W) : (int)(p / a.W);
        float m[kLpl];
        msg(h, horiz ? line : s, horiz ? s : line, dir, m);
        const uint32_t off = (uint32_t)(((p + step_q) * M + x0) * sizeof(float));
        walk_store(out_r, live ? off : kWalkDrop, m);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < kLpl; ++i) carry[i] = m[i];
    }
    __builtin_amdgcn_s_waitcnt(0);  // nothing in flight at exit
}

// kSumF32: the float32 arithmetic of the synchronous and checkerboard
// kernels (sum_message_f), register windows and M = 4G only.
template <int G, int TW, int MODE, int KIND, bool FULL>
__global__ __launch_bounds__(kSweepBlock) void sweep_pass_kernel(UpdateArgs a) {
    static_assert(MODE != kSumF32 || (KIND == kSweepReg && FULL), "float32 sweeps: register windows, M = 4G");
    using HT = typename std::conditional<MODE == kSumF32, float, double>::type;
    constexpr int CAP = G * kLpl;
    extern __shared__ double lds_d[];
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int x0 = pos * kLpl;
    constexpr bool full = FULL;

    // tables in LDS for the LDS-window and dense forms
    double* dtab = lds_d;                                    // kSweepLds sum: w(d); dense sum: f(d)
    float* tab = reinterpret_cast<float*>(lds_d + kMaxTab);  // kSweepLds max: f(d)
    double* Fd = lds_d + kMaxTab;                            // dense sum: F[M][CAP]
    float* F = reinterpret_cast<float*>(lds_d);              // dense max: F[M][CAP]
    double* hs = nullptr;
    if constexpr (KIND == kSweepLds) {
        for (int i = threadIdx.x; i < kMaxTab; i += kSweepBlock) {
            if constexpr (MODE == kSum) dtab[i] = weight_d(a, i);
            else tab[i] = a.tab[i];
        }
        hs = reinterpret_cast<double*>(tab + kMaxTab) + grp * CAP;
        __syncthreads();
    } else if constexpr (KIND == kSweepDense) {
        if constexpr (MODE == kSum) {
            for (int d = threadIdx.x; d < kMaxTab; d += kSweepBlock) dtab[d] = d <= a.T ? exp(-a.alpha_d * d) : 0.0;
            __syncthreads();
            for (int i = threadIdx.x; i < a.M * CAP; i += kSweepBlock) {
                const int x = i / CAP, y = i - x * CAP;
                const int d = x > y ? x - y : y - x;
                Fd[i] = (y >= a.M) ? 0.0 : (d <= a.T ? dtab[d] : a.fbar_d);
            }
            hs = Fd + a.M * CAP + grp * CAP;
        } else {
            for (int i = threadIdx.x; i < a.M * CAP; i += kSweepBlock) {
                const int x = i / CAP, y = i - x * CAP;
                const int d = x > y ? x - y : y - x;
                F[i] = (y >= a.M) ? 0.0f : (d <= a.T ? a.tab[d] : a.fbar);
            }
            hs = reinterpret_cast<double*>(F + a.M * CAP) + grp * CAP;
        }
        __syncthreads();
    }

    auto msg = [&](const HT (&h)[kLpl], int, int, int, float (&m)[kLpl]) {
        if constexpr (MODE == kSumF32) {
            sum_message_f<G, TW>(h, a.tab, a.fbar, pos, a.M, x0, full, m);
        } else if constexpr (KIND == kSweepRegEq10) {
            max_message_eq10_d<G, TW>(h, a.tab, a.fbar, a.T, pos, a.M, x0, full, lds_d + grp * eq10_row_doubles(G), m);
        } else if constexpr (KIND == kSweepReg) {
            if constexpr (MODE == kSum) sum_message_d<G, TW>(h, a.dtab, a.fbar_d, pos, a.M, x0, full, m);
            else max_message_d<G, TW>(h, a.tab, a.fbar, pos, a.M, x0, full, m);
        } else {
#pragma unroll
            for (int i = 0; i < kLpl; ++i) hs[x0 + i] = h[i];
            __syncthreads();
            double u[kLpl];
            if constexpr (MODE == kSum) {
                if constexpr (KIND == kSweepLds) {
                    double s = (h[0] + h[1]) + (h[2] + h[3]);
                    s = group_sum_d<G>(s);
                    const double base = a.fbar_d * s;
#pragma unroll
                    for (int i = 0; i < kLpl; ++i) {
                        const int y = x0 + i;
                        const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
                        double acc = base;
                        for (int x = lo; x <= hi; ++x) acc = fma(dtab[x > y ? x - y : y - x], hs[x], acc);
                        u[i] = acc;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < kLpl; ++i) u[i] = 0.0;
                    for (int x = 0; x < a.M; ++x) {
                        const double hx = hs[x];
#pragma unroll
                        for (int i = 0; i < kLpl; ++i) u[i] = fma(Fd[x * CAP + x0 + i], hx, u[i]);
                    }
                }
            } else {
                if constexpr (KIND == kSweepLds) {
                    const double base = (double)a.fbar * group_max_d<G>(fmax(fmax(h[0], h[1]), fmax(h[2], h[3])));
#pragma unroll
                    for (int i = 0; i < kLpl; ++i) {
                        const int y = x0 + i;
                        const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
                        double acc = base;
                        for (int x = lo; x <= hi; ++x) acc = fmax(acc, (double)tab[x > y ? x - y : y - x] * hs[x]);
                        u[i] = acc;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < kLpl; ++i) u[i] = 0.0;
                    for (int x = 0; x < a.M; ++x) {
                        const double hx = hs[x];
#pragma unroll
                        for (int i = 0; i < kLpl; ++i) u[i] = fmax(u[i], (double)F[x * CAP + x0 + i] * hx);
                    }
                }
            }
            normalise_d<G>(u, a.M, x0, full, m);
            __syncthreads();  // every group done reading hs before the next step writes it
        }
    };
    if constexpr (FULL && KIND == kSweepReg) {
        if ((uint64_t)a.N * a.M * sizeof(float) <= (uint64_t(1) << 31)) {
            sweep_walk_staged<G, HT>(a, msg);
            return;
        }
    }
    sweep_walk<G, FULL, HT>(a, msg);
}

}  // namespace bpk
