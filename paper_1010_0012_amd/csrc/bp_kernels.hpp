// Kernel templates of the grid BP library.  Instantiated and launched from
// the bp_launch_*.hip translation units; declared for the host side in
// bp_launch.hpp.
#pragma once

#include "bp_device.hpp"

namespace bpk {

// Window gather for a pixel group of G lanes: win[(K-J)*4 + i] <- label
// (pos-J)*4 + i and win[(K+J)*4 + i] <- label (pos+J)*4 + i, J = 1..K, 0 for
// lanes outside the group.  The DPP control is an immediate, hence the
// compile-time recursion; wide groups chain one-lane shifts.
template <int G, int K, int J>
__device__ __forceinline__ void fill_window(const float (&h)[kLpl], float (&win)[(2 * K + 1) * kLpl],
                                            int pos, float (&lo)[kLpl], float (&hi)[kLpl]) {
    if constexpr (J <= K) {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            if constexpr (G <= 16) {
                lo[i] = from_lower<G, J>(h[i], pos);
                hi[i] = from_upper<G, J>(h[i], pos);
            } else {
                lo[i] = lower1<G>(lo[i], pos);
                hi[i] = upper1<G>(hi[i], pos);
            }
            win[(K - J) * kLpl + i] = lo[i];
            win[(K + J) * kLpl + i] = hi[i];
        }
        fill_window<G, K, J + 1>(h, win, pos, lo, hi);
    }
}

// ------------------------------------------------ sparse O(mM) update ----
// One message p -> q with the paper's trick.
//   sum (Eq. 7):  u(y) = fbar * S + sum_{|d| <= T} (f(d) - fbar) * h(y + d),
//                 S = sum_x h(x), computed once per message;
//   max (Eq. 11): u(y) = max(fbar * Hm, max_{|d| <= T} f(d) * h(y + d)),
//                 Hm = max_x h(x), computed once per message.
// The window lives in registers: this lane's 4 labels plus the labels of
// K = ceil(TW / 4) neighbouring lanes on each side (gathers that no tap uses
// are dead code).  Labels outside the group read 0, which is also the clip
// at the ends of the label range (Nbd(y) stops at 0 and M-1).  A variant
// compiled for TW >= T runs the taps T < |d| <= TW with weight 0, so
// rounding TW up changes no result.
template <int TW>
constexpr int window_k() { return (TW + kLpl - 1) / kLpl; }

// Symmetric banded window: u[i] = base + sum_{|d| <= TW} tab[|d|] * v(y_i + d)
// (sum) or max(base, max tab[|d|] * v(y_i + d)) (max).
template <int G, int TW, int MODE>
__device__ __forceinline__ void window_apply(const float (&v)[kLpl], const float* tab, float base,
                                             int pos, float (&u)[kLpl]) {
    constexpr int K = window_k<TW>();
    static_assert(K < G, "window wider than the pixel group");
    constexpr int NW = (2 * K + 1) * kLpl;
    float win[NW];
    float lo[kLpl], hi[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        win[K * kLpl + i] = v[i];
        lo[i] = hi[i] = v[i];
    }
    fill_window<G, K, 1>(v, win, pos, lo, hi);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        float acc = base;
#pragma unroll
        for (int d = -TW; d <= TW; ++d) {
            const float w = tab[d < 0 ? -d : d];
            const float x = win[K * kLpl + i + d];
            if constexpr (MODE == kSum) acc = fmaf(w, x, acc);
            else acc = fmaxf(acc, w * x);
        }
        u[i] = acc;
    }
}

// fill_window for double label vectors.
template <int G, int K, int J>
__device__ __forceinline__ void fill_window_d(const double (&h)[kLpl], double (&win)[(2 * K + 1) * kLpl],
                                              int pos, double (&lo)[kLpl], double (&hi)[kLpl]) {
    if constexpr (J <= K) {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            if constexpr (G <= 16) {
                lo[i] = from_lower_d<G, J>(h[i], pos);
                hi[i] = from_upper_d<G, J>(h[i], pos);
            } else {
                lo[i] = lower1_d<G>(lo[i], pos);
                hi[i] = upper1_d<G>(hi[i], pos);
            }
            win[(K - J) * kLpl + i] = lo[i];
            win[(K + J) * kLpl + i] = hi[i];
        }
        fill_window_d<G, K, J + 1>(h, win, pos, lo, hi);
    }
}

// Sum-product window in double: u[i] = base + sum_{|d| <= TW} dtab[|d|] *
// v(y_i + d) with double weights and double h, so the only roundings are the
// double FMAs.  (A float32 h, or float32 weights or accumulation, lose
// relative precision where messages are tiny -- fbar = 0 drives entries to
// zero -- and on ill-conditioned loopy grids.)
template <int G, int TW>
__device__ __forceinline__ void window_sum_d(const double (&v)[kLpl], const double* dtab, double base,
                                             int pos, double (&u)[kLpl]) {
    constexpr int K = window_k<TW>();
    static_assert(K < G, "window wider than the pixel group");
    constexpr int NW = (2 * K + 1) * kLpl;
    double win[NW];
    double lo[kLpl], hi[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        win[K * kLpl + i] = v[i];
        lo[i] = hi[i] = v[i];
    }
    fill_window_d<G, K, 1>(v, win, pos, lo, hi);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        double acc = base;
#pragma unroll
        for (int d = -TW; d <= TW; ++d) acc = fma(dtab[d < 0 ? -d : d], win[K * kLpl + i + d], acc);
        u[i] = acc;
    }
}

// One sum-product message (Eq. 7) in double: S = sum h once per message,
// the window, Z and the normalisation in double, m rounded once to float.
template <int G, int TW>
__device__ __forceinline__ void sum_message_d(const double (&h)[kLpl], const double* dtab, double fbar, int pos,
                                              int M, int x0, bool full, float (&m)[kLpl]) {
    double s = (h[0] + h[1]) + (h[2] + h[3]);
    s = group_sum_d<G>(s);
    double u[kLpl];
    window_sum_d<G, TW>(h, dtab, fbar * s, pos, u);
    normalise_d<G>(u, M, x0, full, m);
}

// Max-product window in double: u[i] = max(base, max_{|d| <= TW} tab[|d|] *
// v(y_i + d)), each product of the float32 f(d) and the double h rounded
// once in double.
template <int G, int TW>
__device__ __forceinline__ void window_max_d(const double (&v)[kLpl], const float* tab, double base,
                                             int pos, double (&u)[kLpl]) {
    constexpr int K = window_k<TW>();
    static_assert(K < G, "window wider than the pixel group");
    constexpr int NW = (2 * K + 1) * kLpl;
    double win[NW];
    double lo[kLpl], hi[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        win[K * kLpl + i] = v[i];
        lo[i] = hi[i] = v[i];
    }
    fill_window_d<G, K, 1>(v, win, pos, lo, hi);
    // f(d) = f(-d) >= 0 and rounding is monotone, so fl(f * max(a, b)) =
    // max(fl(f * a), fl(f * b)): the two taps at +-d share one product (the
    // same bits as taking every tap separately, with 3T+2 instead of 4T+2
    // double operations per label).
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        double acc = fmax(base, (double)tab[0] * win[K * kLpl + i]);
#pragma unroll
        for (int d = 1; d <= TW; ++d)
            acc = fmax(acc, (double)tab[d] * fmax(win[K * kLpl + i - d], win[K * kLpl + i + d]));
        u[i] = acc;
    }
}

// One max-product message (Eq. 11) in double: Hm = max h once per message,
// the window, Z and the normalisation in double, m rounded once to float.
// The max of exact-to-rounding products equals Eq. 9's max bit for bit when
// f >= fbar (rounding is monotone), so the dense kernel, doing the same in
// double, returns the same bits.
template <int G, int TW>
__device__ __forceinline__ void max_message_d(const double (&h)[kLpl], const float* tab, float fbar, int pos,
                                              int M, int x0, bool full, float (&m)[kLpl]) {
    double hm = fmax(fmax(h[0], h[1]), fmax(h[2], h[3]));
    hm = group_max_d<G>(hm);
    double u[kLpl];
    window_max_d<G, TW>(h, tab, (double)fbar * hm, pos, u);
    normalise_d<G>(u, M, x0, full, m);
}

// Eq. 10 for the window potential (some f(d) < fbar): u(y) = max(max over
// |d| <= T of f(d) h(y+d), fbar * max over |x - y| > T of h(x)).  The
// complement maximum is max(P(y - T - 1), S(y + T + 1)), P and S the prefix
// and suffix maxima of h over the labels (0 past either end).  The lanes'
// block maxima go through the group's LDS row (G reads per lane for the
// scans), then P and S go through it for the shifted reads.  Both parts are
// maxima of the rounded products Eq. 9's max takes (fbar * max h = max of
// fbar * h, rounding being monotone), so the result equals the dense
// kernel's bit for bit.
constexpr int eq10_row_doubles(int G) { return G + 2 * G * kLpl; }

// Hillis-Steele max scans over a group of G <= 16 lanes, steps K, 2K, ...:
// pre ends as the max over lanes 0..pos, suf over lanes pos..G-1.
template <int G, int K>
__device__ __forceinline__ void scan_max_d(double& pre, double& suf, int pos) {
    if constexpr (K < G) {
        const double lo = from_lower_d<G, K>(pre, pos);
        const double hi = from_upper_d<G, K>(suf, pos);
        pre = fmax(pre, lo);
        suf = fmax(suf, hi);
        scan_max_d<G, 2 * K>(pre, suf, pos);
    }
}

template <int G, int TW>
__device__ __forceinline__ void max_message_eq10_d(const double (&h)[kLpl], const float* tab, float fbar, int T,
                                                   int pos, int M, int x0, bool full, double* row, float (&m)[kLpl]) {
    constexpr int CAP = G * kLpl;
    double* lm = row;     // [G] block maxima
    double* P = row + G;  // [CAP] prefix maxima
    double* S = P + CAP;  // [CAP] suffix maxima
    wave_sync();          // the previous message is done with the row
    const double bm = fmax(fmax(h[0], h[1]), fmax(h[2], h[3]));
    double before = 0.0, after = 0.0;  // max of the block maxima of the lanes below / above
    if constexpr (G <= 16) {
        // inclusive max scans up and down the group by lane shifts (0 past
        // the group's ends), then one more shift for the exclusive ones
        double pre = bm, suf = bm;
        scan_max_d<G, 1>(pre, suf, pos);
        before = from_lower_d<G, 1>(pre, pos);
        after = from_upper_d<G, 1>(suf, pos);
    } else {
        lm[pos] = bm;
        wave_sync();
        for (int j = 0; j < G; ++j) {
            const double v = lm[j];
            if (j < pos) before = fmax(before, v);
            if (j > pos) after = fmax(after, v);
        }
    }
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        before = fmax(before, h[i]);
        P[x0 + i] = before;
    }
#pragma unroll
    for (int i = kLpl - 1; i >= 0; --i) {
        after = fmax(after, h[i]);
        S[x0 + i] = after;
    }
    wave_sync();
    double u[kLpl];
    window_max_d<G, TW>(h, tab, 0.0, pos, u);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        const int lo = x0 + i - T - 1, hi = x0 + i + T + 1;
        const double out = fmax(lo >= 0 ? P[lo] : 0.0, hi < M ? S[hi] : 0.0);
        u[i] = fmax(u[i], (double)fbar * out);
    }
    normalise_d<G>(u, M, x0, full, m);
}

// Double weights w(d) = f(d) - fbar for d <= T (f(d) = exp(-alpha d)) built
// on the device, for kernels whose windows reach past the argument table.
__device__ __forceinline__ double weight_d(const UpdateArgs& a, int d) {
    return d <= a.T ? exp(-a.alpha_d * d) - a.fbar_d : 0.0;
}

// Group-wide sum (or max) of a 4-per-lane vector; same bits on every lane.
template <int G, int MODE>
__device__ __forceinline__ float group_total(const float (&v)[kLpl]) {
    float s = v[0];
#pragma unroll
    for (int i = 1; i < kLpl; ++i) s = (MODE == kSum) ? s + v[i] : fmaxf(s, v[i]);
    return group_reduce<MODE, G>(s);
}

// ------------------------------------- FP32 arithmetic (sum-product) ----
// The Eq. 7 message with h, S, the window, Z and the normalisation all in
// float32 (the BP_ARITH_F32 setting of a grid): one FP32 FMA per tap, one DPP
// move per shifted value and no conversions, against the double path's two
// moves per value and the conversions in and out.  Every step rounds to
// float32, so a message carries a few roundings instead of one; sum-product
// contracts them (the synchronous and checkerboard kernels use it; the
// results agree with the double path to rounding, not bit for bit).
__device__ __forceinline__ void sender_h_f(const float (&g)[kLpl], const float (&ma)[kLpl], const float (&mb)[kLpl],
                                           const float (&mc)[kLpl], float (&h)[kLpl]) {
#pragma unroll
    for (int i = 0; i < kLpl; ++i) h[i] = ((g[i] * ma[i]) * mb[i]) * mc[i];
}

// 1/z from the hardware reciprocal and one Newton step (about one ulp).
__device__ __forceinline__ float recip_f(float z) {
    const float r = __builtin_amdgcn_rcpf(z);
    return fmaf(r, fmaf(-z, r, 1.0f), r);
}

template <int G>
__device__ __forceinline__ void normalise_f(float (&u)[kLpl], int M, int x0, bool full, float (&m)[kLpl]) {
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        if (!full && x0 + i >= M) u[i] = 0.0f;
        z += u[i];
    }
    z = group_sum<G>(z);
    const float inv = recip_f(z);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) m[i] = u[i] * inv;
}

// wtab: f(d) - fbar in float32 for d <= T (0 beyond), fbar in float32.
template <int G, int TW>
__device__ __forceinline__ void sum_message_f(const float (&h)[kLpl], const float* wtab, float fbar, int pos, int M,
                                              int x0, bool full, float (&m)[kLpl]) {
    float s = (h[0] + h[1]) + (h[2] + h[3]);
    s = group_sum<G>(s);
    float u[kLpl];
    window_apply<G, TW, kSum>(h, wtab, fbar * s, pos, u);
    normalise_f<G>(u, M, x0, full, m);
}

// Grid-wide update, register window.  One group of G lanes per sending
// pixel; a wave's load and store instructions cover 64/G consecutive pixels.
// EQ10: max-product with Eq. 10 (max_message_eq10_d, one LDS row per group).
template <int G, int TW, int MODE, bool EQ10 = false>
__global__ __launch_bounds__(kBlock) void sparse_update_kernel(UpdateArgs a) {
    extern __shared__ double lds_d[];
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;  // whole groups only: no shuffle reads a retired lane's value
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    PixelInputs in;
    load_pixel(a, px, x0, full, in);
    const size_t plane = (size_t)a.N * a.M;
    if constexpr (MODE == kSumF32) {
        float h[4][kLpl];
        make_h(in, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[kLpl];
            sum_message_f<G, TW>(h[o], a.tab, a.fbar, pos, a.M, x0, full, u);
            store_message(a.out, plane, a.M, a.W, px, o, x0, full, u);
        }
    } else {
        double h[4][kLpl];
        make_h_d(in, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[kLpl];
            if constexpr (MODE == kSum) sum_message_d<G, TW>(h[o], a.dtab, a.fbar_d, pos, a.M, x0, full, u);
            else if constexpr (EQ10)
                max_message_eq10_d<G, TW>(h[o], a.tab, a.fbar, a.T, pos, a.M, x0, full,
                                          lds_d + (threadIdx.x / G) * eq10_row_doubles(G), u);
            else max_message_d<G, TW>(h[o], a.tab, a.fbar, pos, a.M, x0, full, u);
            store_message(a.out, plane, a.M, a.W, px, o, x0, full, u);
        }
    }
}

// -------------------------------- two synchronous iterations per launch ----
// Iteration t+1's outgoing messages of p need only p's unary and the four
// messages its neighbours send it at iteration t, and each of those needs
// only its sender's unary and three of the sender's inbox rows.  So one
// group computes p's four incoming messages from the neighbours' inputs
// (receiver side: every message of iteration t is still computed exactly
// once), then p's four outgoing messages, and iteration t's messages never
// reach HBM: a launch reads the unary and the inbox and writes the outbox
// once for two iterations.  The neighbours' rows are read up to four times,
// from L2: the launches keep a pixel's neighbours on its own XCD (its own
// L2) -- sparse_update2_kernel gives each XCD a contiguous band of rows, the
// row-block launch whole column strips.  The arithmetic of both iterations
// is that of sparse_update_kernel, so the results equal two of its launches
// bit for bit.

// h of the message a sender sends towards o (Eq. 5, the factor order of
// make_h_d): horizontal targets ((g mU) mD) m_{opp(o)}, vertical ones
// ((g mL) mR) m_{opp(o)}.
__device__ __forceinline__ void sender_h_d(const float (&g)[kLpl], const float (&ma)[kLpl], const float (&mb)[kLpl],
                                           const float (&mc)[kLpl], double (&h)[kLpl]) {
#pragma unroll
    for (int i = 0; i < kLpl; ++i) h[i] = (((double)g[i] * ma[i]) * mb[i]) * mc[i];
}

// Workgroups per XCD band: the hardware deals workgroups to the 8 XCDs in
// turn, so block b runs on XCD b mod 8; logical block (b mod 8) * per + b / 8
// gives XCD x the contiguous range [x * per, (x + 1) * per).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_band_block(int b, int per) { return (b % kXcds) * per + b / kXcds; }

// A read-only row of ones: a missing inbox row is loaded from here instead
// of being replaced after the load (one address select per row instead of
// one value select per label).
struct OnesRow {
    float v[kMaxTab];
    constexpr OnesRow() : v() {
        for (int i = 0; i < kMaxTab; ++i) v[i] = 1.0f;
    }
};
static __device__ OnesRow kOnesRow = OnesRow();  // never written

// One message in double from explicit tables (sum: dtab = f - fbar in
// double, fbar_d; max: tab = float32 f, fbar).
template <int G, int TW, int MODE>
__device__ __forceinline__ void message_d(const double (&h)[kLpl], const double* dtab, double fbar_d,
                                          const float* tab, float fbar, int pos, int M, int x0, bool full,
                                          float (&m)[kLpl]) {
    if constexpr (MODE == kSum) sum_message_d<G, TW>(h, dtab, fbar_d, pos, M, x0, full, m);
    else max_message_d<G, TW>(h, tab, fbar, pos, M, x0, full, m);
}

// One first-iteration message into a receiver: rows are the sender's unary
// and the three inbox rows its message uses ({g, the two partial-product
// rows, the far-side row}); has says whether the sender exists (the factor 1
// where it does not).
template <int G, int TW, int MODE>
__device__ __forceinline__ void pair_first(const float (&rows)[4][kLpl], bool has, int pos, int M, bool full,
                                           const double* dtab, double fbar_d, const float* tab, float fbar,
                                           float (&m)[kLpl]) {
    const int x0 = pos * kLpl;
    if constexpr (MODE == kSumF32) {
        float h[kLpl];
        sender_h_f(rows[0], rows[1], rows[2], rows[3], h);
        sum_message_f<G, TW>(h, tab, fbar, pos, M, x0, full, m);
    } else {
        double h[kLpl];
        sender_h_d(rows[0], rows[1], rows[2], rows[3], h);
        message_d<G, TW, MODE>(h, dtab, fbar_d, tab, fbar, pos, M, x0, full, m);
    }
#pragma unroll
    for (int i = 0; i < kLpl; ++i) m[i] = has ? m[i] : 1.0f;
}

// The second iteration, sender side: p's four outgoing messages from its
// unary (mid.g) and the first-iteration messages into it (mid.m).
template <int G, int TW, int MODE, bool FULL, class PutOut>
__device__ __forceinline__ void pair_second(const PixelInputs& mid, int pos, int M, const double* dtab, double fbar_d,
                                            const float* tab, float fbar, PutOut put_out) {
    const int x0 = pos * kLpl;
    if constexpr (MODE == kSumF32) {
        float h[4][kLpl];
        make_h(mid, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[kLpl];
            sum_message_f<G, TW>(h[o], tab, fbar, pos, M, x0, FULL, u);
            put_out(o, u);
        }
    } else {
        double h[4][kLpl];
        make_h_d(mid, h);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float u[kLpl];
            message_d<G, TW, MODE>(h[o], dtab, fbar_d, tab, fbar, pos, M, x0, FULL, u);
            put_out(o, u);
        }
    }
}

// The arithmetic of both iterations for one receiver p: rows[k] are the
// unary and the three inbox rows of the neighbour in direction k that its
// message to p uses, gp is p's unary, has[k] whether that neighbour exists.
// put_mid(k, m) takes each first-iteration message into p (the factor 1
// where there is no neighbour), put_out(o, u) each second-iteration message
// p sends.
template <int G, int TW, int MODE, bool FULL, class PutMid, class PutOut>
__device__ __forceinline__ void pair_compute(const float (&rows)[4][4][kLpl], const float (&gp)[kLpl],
                                             const bool (&has)[4], int pos, int M, const double* dtab,
                                             double fbar_d, const float* tab, float fbar, PutMid put_mid,
                                             PutOut put_out) {
    PixelInputs mid;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pair_first<G, TW, MODE>(rows[k], has[k], pos, M, FULL, dtab, fbar_d, tab, fbar, mid.m[k]);
        put_mid(k, mid.m[k]);
    }
#pragma unroll
    for (int i = 0; i < kLpl; ++i) mid.g[i] = gp[i];
    pair_second<G, TW, MODE, FULL>(mid, pos, M, dtab, fbar_d, tab, fbar, put_out);
}

// Inbox rows of the neighbour q in direction k that q's message to p uses:
// q sees p in direction opposite(k) and leaves out its own row from p; the
// partial product pairs the two rows across that axis.
__device__ __forceinline__ void pair_sources(int k, int (&src)[3]) {
    const int o = opposite(k);  // direction of p seen from q
    const int ka = (o == kLeft || o == kRight) ? kUp : kLeft;
    src[0] = ka;
    src[1] = ka + 1;
    src[2] = opposite(o);
}

// Both iterations for one pixel px of an H x W grid (in -> out); with
// mid_out, the first iteration's messages into px are stored there too
// (px's own inbox slots, coalesced).  FULL:
// M == 4G, known at compile time so that no load or normalisation carries a
// branch.  Loads are unconditional: a missing neighbour (or a missing row of
// a neighbour's inbox) reads a valid row and is replaced by the factor 1,
// which keeps every load of the pixel in one basic block.
template <int G, int TW, int MODE, bool FULL>
__device__ __forceinline__ void pair_pixel(const float* g, const float* in, float* out, float* mid_out, int H, int W,
                                           int M, const Pixel& px, int pos, const double* dtab, double fbar_d,
                                           const float* tab, float fbar) {
    const int x0 = pos * kLpl;
    const size_t plane = (size_t)H * W * M;
    float rows[4][4][kLpl];  // [k][g, the two partial-product rows, the opposite row]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int src[3];
        pair_sources(k, src);
        const int qr = px.has[k] ? px.r + (k == kUp ? -1 : k == kDown ? 1 : 0) : px.r;
        const int qc = px.has[k] ? px.c + (k == kLeft ? -1 : k == kRight ? 1 : 0) : px.c;
        const bool qhas[4] = {qc > 0, qc + 1 < W, qr > 0, qr + 1 < H};
        const size_t qoff = ((size_t)qr * W + qc) * M;
        load_labels<false>(g + qoff, x0, M, FULL, rows[k][0], 0.0f);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float* row = qhas[src[j]] ? in + src[j] * plane + qoff : kOnesRow.v;
            load_labels<false>(row, x0, M, FULL, rows[k][j + 1], 1.0f);
        }
    }
    float gp[kLpl];
    load_labels<false>(g + (size_t)px.p * M, x0, M, FULL, gp, 0.0f);
    pair_compute<G, TW, MODE, FULL>(
        rows, gp, px.has, pos, M, dtab, fbar_d, tab, fbar,
        [&](int k, const float (&m)[kLpl]) {
            if (mid_out && px.has[k]) store_labels<kMsgNT>(mid_out + k * plane + (size_t)px.p * M, x0, M, FULL, m);
        },
        [&](int o, const float (&u)[kLpl]) { store_message(out, plane, M, W, px, o, x0, FULL, u); });
}

// Global-memory byte pointers.  A float4 at a 32-bit byte offset from a
// uniform base: the access takes its base from scalar registers and its
// offset from one VGPR, with no 64-bit address arithmetic per row.
typedef const char __attribute__((address_space(1)))* gcptr;
typedef char __attribute__((address_space(1)))* gptr;

// A uniform pointer, held in scalar registers as such: without this the
// compiler may fold a uniform plane offset into the per-lane address and
// form 64-bit addresses in VGPRs again.
template <typename P>
__device__ __forceinline__ P uniform_ptr(P p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ v4f ld_off(gcptr base, uint32_t off) {
    return *(const v4f __attribute__((address_space(1)))*)(base + off);
}
__device__ __forceinline__ void st_off_nt(gptr base, uint32_t off, const float (&v)[kLpl]) {
    __builtin_nontemporal_store(v4f{v[0], v[1], v[2], v[3]}, (v4f __attribute__((address_space(1)))*)(base + off));
}
__device__ __forceinline__ void unpack(v4f t, float (&v)[kLpl]) {
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}

// pair_pixel for M = 4G and a pixel at least two rows and two columns away
// from every grid border: every one of the seventeen rows exists and all
// four outgoing messages are stored, so no row is replaced and no store is
// conditional.  voff is the byte offset of p's label row plus this lane's
// 16 bytes; plane_b (bytes of one inbox plane) and row_b (bytes of one grid
// row of label rows) are below 2^32, so every offset is 32-bit.  The same
// pair_compute as pair_pixel: the same bits.
template <int G, int TW, int MODE>
__device__ __forceinline__ void pair_pixel_inner(gcptr gb, gcptr ib, gptr ob, gptr mb, uint32_t plane_b,
                                                 uint32_t row_b, uint32_t voff, int pos, const double* dtab,
                                                 double fbar_d, const float* tab, float fbar) {
    constexpr uint32_t lab_b = 16u * G;  // bytes of one label row
    const uint32_t q_off[4] = {voff - lab_b, voff + lab_b, voff - row_b, voff + row_b};
    gcptr ib_plane[4];
    gptr ob_plane[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ib_plane[k] = uniform_ptr(ib + (size_t)k * plane_b);
        ob_plane[k] = uniform_ptr(ob + (size_t)k * plane_b);
    }
    float rows[4][4][kLpl];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int src[3];
        pair_sources(k, src);
        unpack(ld_off(gb, q_off[k]), rows[k][0]);
#pragma unroll
        for (int j = 0; j < 3; ++j) unpack(ld_off(ib_plane[src[j]], q_off[k]), rows[k][j + 1]);
    }
    float gp[kLpl];
    unpack(ld_off(gb, voff), gp);
    const bool all[4] = {true, true, true, true};
    pair_compute<G, TW, MODE, true>(
        rows, gp, all, pos, 4 * G, dtab, fbar_d, tab, fbar,
        [&](int k, const float (&m)[kLpl]) {
            if (mb) st_off_nt(uniform_ptr(mb + (size_t)k * plane_b), voff, m);
        },
        [&](int o, const float (&u)[kLpl]) { st_off_nt(ob_plane[opposite(o)], q_off[o], u); });
}

// Synchronous (a.colour < 0): every pixel, two iterations a.in -> a.out,
// the first iteration's state optionally into a.mid.  Checkerboard pair
// (a.colour = c): the passes of colour 1 - c and then c, as one launch over
// the pixels of colour c: each forms the messages its (colour 1 - c)
// neighbours send it and stores them in its own inbox in a.out (a.mid ==
// a.out), then sends its own into its neighbours' inboxes in a.out.  Every
// inbox slot of a.out is written (colour-c pixels hear only from colour
// 1 - c and vice versa), and every value equals the in-place passes'.
template <int G, int TW, int MODE, bool FULL>
__global__ __launch_bounds__(kBlock) void sparse_update2_kernel(UpdateArgs a, int per) {
    const int b = xcd_band_block(blockIdx.x, per);
    const int pos = threadIdx.x & (G - 1);
    const int slot = (b * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;  // whole groups only
    pair_pixel<G, TW, MODE, FULL>(a.g, a.in, a.out, a.mid, a.H, a.W, a.M, px, pos, a.dtab, a.fbar_d, a.tab, a.fbar);
}

// Both iterations for pixel (r, c) of an H x W grid with M = 4G whose inbox
// plane is below 2^32 bytes, as the row-block launches run them: a wave
// whose pixels all lie two or more pixels inside the grid takes
// pair_pixel_inner, any other wave pair_pixel (the same bits).
template <int G, int TW, int MODE>
__device__ __forceinline__ void pair_rows_pixel(const float* g, const float* in, float* out, float* mid, int H, int W,
                                                int r, int c, int pos, const double* dtab, double fbar_d,
                                                const float* tab, float fbar) {
    const int p = r * W + c;
    const bool inner = r >= 2 && r + 2 < H && c >= 2 && c + 2 < W;
    if (__builtin_amdgcn_ballot_w64(!inner) == 0) {
        const uint32_t plane_b = (uint32_t)(H * W) * (16u * G);
        const uint32_t row_b = (uint32_t)W * (16u * G);
        const uint32_t voff = (uint32_t)p * (16u * G) + (uint32_t)pos * 16u;
        pair_pixel_inner<G, TW, MODE>((gcptr)g, (gcptr)in, (gptr)out, (gptr)mid, plane_b, row_b, voff, pos, dtab,
                                      fbar_d, tab, fbar);
    } else {
        Pixel px;
        px.r = r;
        px.c = c;
        px.p = p;
        px.ok = true;
        px.has[kLeft] = c > 0;
        px.has[kRight] = c + 1 < W;
        px.has[kUp] = r > 0;
        px.has[kDown] = r + 1 < H;
        pair_pixel<G, TW, MODE, true>(g, in, out, mid, H, W, 4 * G, px, pos, dtab, fbar_d, tab, fbar);
    }
}

// The same launch for M = 4G when an inbox plane is below 2^32 bytes, with
// workgroups that each cover kBlock/G consecutive pixels (or colour slots) of
// one grid row: the row and column come from the workgroup index in scalar
// registers (no per-lane division), and a wave whose pixels all lie two or
// more pixels inside the grid runs pair_pixel_inner.  gx = workgroups per
// row, padded to gxp, a multiple of the XCD count (the padding exits at
// once): in launch order workgroup b runs on XCD b mod 8, so each XCD holds
// the same column strips in every row, the rows above and below a pixel are
// read through that XCD's own L2, and all XCDs sweep the grid top to bottom
// together.  With per > 0 the workgroups are remapped as in
// sparse_update2_kernel instead (gxp = gx), so that each XCD holds a
// contiguous band of rows (at 480 x 640 x 64 that measured 6% slower);
// with per < 0 XCD x holds the contiguous column blocks [x gxp/8, (x+1)
// gxp/8) of every row, one wide strip, so that only the strips' edge
// columns are read by two XCDs.
template <int G, int TW, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_update2_rows_kernel(UpdateArgs a, int gxp, int gx, int per) {
    constexpr int PPB = kBlock / G;
    int r, cb;
    if (per < 0) {
        const int wide = gxp / kXcds;  // column blocks per XCD strip
        const int x = (int)blockIdx.x % kXcds, k = (int)blockIdx.x / kXcds;
        r = k / wide;
        cb = x * wide + (k - r * wide);
    } else {
        const int b = per > 0 ? xcd_band_block((int)blockIdx.x, per) : (int)blockIdx.x;
        r = b / gxp;
        cb = b - r * gxp;
    }
    if (cb >= gx) return;  // padding: whole workgroup
    const int j = cb * PPB + (int)(threadIdx.x / G);
    const int pos = threadIdx.x & (G - 1);
    const int c = a.colour < 0 ? j : 2 * j + ((a.colour + r) & 1);
    if (r >= a.H || c >= a.W) return;  // whole groups only
    pair_rows_pixel<G, TW, MODE>(a.g, a.in, a.out, a.mid, a.H, a.W, r, c, pos, a.dtab, a.fbar_d, a.tab, a.fbar);
}

// ------------------------------------- sparse update, runtime window ----
// Same arithmetic for windows wider than the compiled register variants:
// h is staged in LDS per pixel and the compatible states of each y are
// visited with runtime bounds [max(0, y-T), min(M-1, y+T)].
constexpr size_t wide_lds_bytes(int G) {
    return kMaxTab * sizeof(double) + kMaxTab * sizeof(float) + (size_t)(kBlock / G) * G * kLpl * sizeof(double);
}

template <int G, int MODE>
__global__ __launch_bounds__(kBlock) void sparse_update_wide_kernel(UpdateArgs a) {
    extern __shared__ double lds_d[];  // dtab[kMaxTab] (sum), tab[kMaxTab] (max), h[kBlock/G][4G] (double)
    constexpr int CAP = G * kLpl;
    double* dtab = lds_d;
    float* tab = reinterpret_cast<float*>(lds_d + kMaxTab);
    double* lds_h = reinterpret_cast<double*>(tab + kMaxTab);
    for (int i = threadIdx.x; i < kMaxTab; i += kBlock) {
        if constexpr (MODE == kSum) dtab[i] = weight_d(a, i);
        else tab[i] = a.tab[i];
    }
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    PixelInputs in;
    if (px.ok) load_pixel(a, px, x0, full, in); else dummy_pixel(in);
    double h[4][kLpl];
    make_h_d(in, h);
    double* hs = lds_h + grp * CAP;
    __syncthreads();
#pragma unroll 1
    for (int o = 0; o < 4; ++o) {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) hs[x0 + i] = h[o][i];
        __syncthreads();
        // the once-per-message term, then the compatible states of each y
        const double base = MODE == kSum
            ? a.fbar_d * group_sum_d<G>((h[o][0] + h[o][1]) + (h[o][2] + h[o][3]))
            : (double)a.fbar * group_max_d<G>(fmax(fmax(h[o][0], h[o][1]), fmax(h[o][2], h[o][3])));
        double ud[kLpl];
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            const int y = x0 + i;
            const int lo = max(0, y - a.T), hi = min(a.M - 1, y + a.T);
            double acc = base;
            for (int x = lo; x <= hi; ++x) {
                const int d = x > y ? x - y : y - x;
                if constexpr (MODE == kSum) acc = fma(dtab[d], hs[x], acc);
                else acc = fmax(acc, (double)tab[d] * hs[x]);
            }
            ud[i] = acc;
        }
        float u[kLpl];
        normalise_d<G>(ud, a.M, x0, full, u);
        __syncthreads();
        store_message(a.out, (size_t)a.N * a.M, a.M, a.W, px, o, x0, full, u);
    }
}

// ------------------------------------------ dense O(M^2) comparison ----
// Eq. 2 / Eq. 9 as written: u(y) = sum (or max) over every sender label x of
// F[x][y] * h(x), with F the full M x M table (f(|x-y|) inside the window,
// fbar outside) staged in LDS once per workgroup.  h, the precision, the
// normalisation and the store are those of the sparse kernels, so
// max-product results match them bit for bit.
// Workgroups loop over tiles of kBlock/G pixels to amortise the table.
// LDS of the dense kernel: sum-product keeps F in double (with a double
// f(d) table to build it from), max-product in float32; h in double.
// Workgroup size: 128 threads for 32-lane groups keeps the M = 128 double
// table plus h within the 160 KB of LDS.
constexpr int dense_block(int G) { return G >= 32 ? 128 : kBlock; }

constexpr size_t dense_lds_bytes(int G, int M, int mode) {
    const size_t hbytes = (size_t)dense_block(G) * kLpl * 4 * sizeof(double);
    return mode == kSum ? kMaxTab * sizeof(double) + (size_t)M * G * kLpl * sizeof(double) + hbytes
                        : (size_t)M * G * kLpl * sizeof(float) + hbytes;
}

template <int G, int MODE>
__global__ __launch_bounds__(dense_block(G)) void dense_update_kernel(UpdateArgs a) {
    extern __shared__ double lds_d[];
    constexpr int CAP = G * kLpl;
    constexpr int BLK = dense_block(G);
    constexpr int RPB = BLK / G;
    double* Fd = lds_d + kMaxTab;                              // sum: F[M][4G] in double
    float* F = reinterpret_cast<float*>(lds_d);                // max: F[M][4G] in float32
    double* hsd = MODE == kSum ? Fd + a.M * CAP : reinterpret_cast<double*>(F + a.M * CAP);
    if constexpr (MODE == kSum) {
        double* fd = lds_d;                                    // f(d) = exp(-alpha d), d <= T
        for (int d = threadIdx.x; d < kMaxTab; d += BLK) fd[d] = d <= a.T ? exp(-a.alpha_d * d) : 0.0;
        __syncthreads();
        for (int i = threadIdx.x; i < a.M * CAP; i += BLK) {
            const int x = i / CAP, y = i - x * CAP;
            const int d = x > y ? x - y : y - x;
            Fd[i] = (y >= a.M) ? 0.0 : (d <= a.T ? fd[d] : a.fbar_d);
        }
    } else {
        for (int i = threadIdx.x; i < a.M * CAP; i += BLK) {
            const int x = i / CAP, y = i - x * CAP;
            const int d = x > y ? x - y : y - x;
            F[i] = (y >= a.M) ? 0.0f : (d <= a.T ? a.tab[d] : a.fbar);
        }
    }
    const int pos = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int x0 = pos * kLpl;
    const bool full = a.M == CAP;
    const int n_tiles = (a.n_slots + RPB - 1) / RPB;
    double* hgd = hsd + grp * CAP * 4;
    const size_t plane = (size_t)a.N * a.M;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const Pixel px = map_slot(tile * RPB + grp, a);
        PixelInputs in;
        if (px.ok) load_pixel(a, px, x0, full, in); else dummy_pixel(in);
        double h[4][kLpl];
        make_h_d(in, h);
        __syncthreads();  // previous tile done with h (and F built on entry)
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            *reinterpret_cast<double2*>(hgd + (x0 + i) * 4) = make_double2(h[0][i], h[1][i]);
            *reinterpret_cast<double2*>(hgd + (x0 + i) * 4 + 2) = make_double2(h[2][i], h[3][i]);
        }
        __syncthreads();
        double u[4][kLpl];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int i = 0; i < kLpl; ++i) u[o][i] = 0.0;
        for (int x = 0; x < a.M; ++x) {
            const double2 h01 = *reinterpret_cast<const double2*>(hgd + x * 4);
            const double2 h23 = *reinterpret_cast<const double2*>(hgd + x * 4 + 2);
            double f[kLpl];
            if constexpr (MODE == kSum) {
                const double2 f01 = *reinterpret_cast<const double2*>(Fd + x * CAP + x0);
                const double2 f23 = *reinterpret_cast<const double2*>(Fd + x * CAP + x0 + 2);
                f[0] = f01.x; f[1] = f01.y; f[2] = f23.x; f[3] = f23.y;
            } else {
                const float4 fr = *reinterpret_cast<const float4*>(F + x * CAP + x0);
                f[0] = fr.x; f[1] = fr.y; f[2] = fr.z; f[3] = fr.w;
            }
#pragma unroll
            for (int i = 0; i < kLpl; ++i) {
                if constexpr (MODE == kSum) {
                    u[0][i] = fma(f[i], h01.x, u[0][i]);
                    u[1][i] = fma(f[i], h01.y, u[1][i]);
                    u[2][i] = fma(f[i], h23.x, u[2][i]);
                    u[3][i] = fma(f[i], h23.y, u[3][i]);
                } else {
                    // the products and the max as in the sparse kernel, so both
                    // return the same bits
                    u[0][i] = fmax(u[0][i], f[i] * h01.x);
                    u[1][i] = fmax(u[1][i], f[i] * h01.y);
                    u[2][i] = fmax(u[2][i], f[i] * h23.x);
                    u[3][i] = fmax(u[3][i], f[i] * h23.y);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float m[kLpl];
            normalise_d<G>(u[o], a.M, x0, full, m);
            store_message(a.out, plane, a.M, a.W, px, o, x0, full, m);
        }
    }
}

// ------------------------------- dense O(M^2) sum-product, matrix cores ----
// Eq. 2 for M = 32 or 64 (full label rows) as the matrix product it is: the
// u rows of a wave's messages (four per pixel: 16 for M = 64, 32 for M = 32)
// are H F, H the wave's h rows [message][x] and F the M x M table.  The
// products run on v_mfma_f64_16x16x4 (FP64 operands, FP64 accumulation;
// no algebraic shortcut, every F[x][y] h(x) product is formed), 16 messages
// by 16 labels by 4 sender labels per instruction: each lane holds its F
// operands in registers and reads one double of H from LDS per step of four
// instructions.  h, the normalisation and the store are those of the other
// kernels.  The 16 steps are unrolled so that the accumulators stay in the
// matrix registers for the whole product.
// Operand layout of the instruction (measured on gfx950): A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i mod 4),
// element i / 4.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int G>
constexpr size_t dense_mfma_lds_bytes() {
    constexpr int M = 4 * G;
    return ((size_t)kMaxTab + (size_t)(kBlock / 64) * (4 * (64 / G)) * (M + 1)) * sizeof(double);
}

template <int G>
__global__ __launch_bounds__(kBlock) void dense_mfma_kernel(UpdateArgs a) {
    constexpr int M = 4 * G;           // full rows only
    constexpr int MPW = 4 * (64 / G);  // messages per wave
    constexpr int LD = M + 1;          // row stride in doubles (spreads a column over the banks)
    constexpr int KS = M / 4;          // sender-label steps
    constexpr int CT = M / 16;         // 16-label column tiles
    constexpr int RPB = kBlock / G;    // pixels per workgroup tile
    static_assert(MPW % 16 == 0, "whole 16-message batches");
    extern __shared__ double lds_d[];
    double* fd = lds_d;                                       // f(d) = exp(-alpha d), d <= T
    double* rows = fd + kMaxTab + (threadIdx.x / 64) * MPW * LD;  // this wave's [MPW][LD]
    for (int d = threadIdx.x; d < kMaxTab; d += kBlock) fd[d] = d <= a.T ? exp(-a.alpha_d * d) : 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int pos = threadIdx.x & (G - 1);
    const int gw = lane / G;      // pixel group within the wave
    const int x0 = pos * kLpl;
    const int li = lane & 15, lk = lane >> 4;
    // This lane's B operands for every product: F[4t + lk][16c + li], F[x][y]
    // = f(|x - y|) within the window and fbar outside, the same for every
    // tile, so they are formed once and kept in registers (64 doubles at
    // M = 64; read from an LDS copy of F in each product they cost about 2%).
    double bop[KS][CT];
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int x = 4 * t + lk, y = 16 * c + li;
            const int d = x > y ? x - y : y - x;
            bop[t][c] = d <= a.T ? fd[d] : a.fbar_d;
        }
    const int n_tiles = (a.n_slots + RPB - 1) / RPB;
    const size_t plane = (size_t)a.N * M;
    // the next tile's inputs are loaded before this tile's products run
    Pixel px_next = map_slot(blockIdx.x * RPB + (int)(threadIdx.x / G), a);
    PixelInputs in_next;
    if (blockIdx.x < n_tiles && px_next.ok) load_pixel(a, px_next, x0, true, in_next); else dummy_pixel(in_next);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const Pixel px = px_next;
        double h[4][kLpl];
        make_h_d(in_next, h);
        const int nt = tile + gridDim.x;
        px_next = map_slot(nt * RPB + (int)(threadIdx.x / G), a);
        if (nt < n_tiles && px_next.ok) load_pixel(a, px_next, x0, true, in_next); else dummy_pixel(in_next);
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int i = 0; i < kLpl; ++i) rows[(gw * 4 + o) * LD + x0 + i] = h[o][i];
        wave_sync();
#pragma unroll
        for (int nb = 0; nb < MPW / 16; ++nb) {
            v4d acc[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
            const double* arow = rows + (nb * 16 + li) * LD + lk;
            // fully unrolled: the accumulators stay in the matrix registers (a
            // loop back-edge moved them to VGPRs and back, each move waiting for
            // the last product: 270 -> 254 us per iteration at 480x640x64)
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const double av = arow[4 * t];
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bop[t][c], acc[c], 0, 0, 0);
            }
            wave_sync();  // every read of this batch's h rows is done
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) rows[(nb * 16 + 4 * r + lk) * LD + 16 * c + li] = acc[c][r];
        }
        wave_sync();
        double u[4][kLpl];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int i = 0; i < kLpl; ++i) u[o][i] = rows[(gw * 4 + o) * LD + x0 + i];
        wave_sync();  // the rows are free for the next tile
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float m[kLpl];
            normalise_d<G>(u[o], M, x0, true, m);
            store_message(a.out, plane, M, a.W, px, o, x0, true, m);
        }
    }
}

// ------------------------------------------------------------ readout ----
// Eq. 3: b = g * product of all incoming messages, normalised (belief_d);
// MAP label = argmax of the normalised float32 beliefs, lowest label on ties.
template <int G>
__device__ __forceinline__ void readout_pixel(const PixelInputs& in, int M, int x0, bool full,
                                              float* beliefs_row, int* label) {
    float b[kLpl];
    belief_d<G>(in, M, x0, full, b);
    float best = -1.0f;
    int arg = 0x7fffffff;
#pragma unroll
    for (int i = 0; i < kLpl; ++i)
        if (x0 + i < M && b[i] > best) { best = b[i]; arg = x0 + i; }
    if (beliefs_row) store_labels<false>(beliefs_row, x0, M, full, b);
    if (label) {
        group_argmax<G>(best, arg);
        if (x0 == 0) *label = arg;
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void readout_kernel(UpdateArgs a, float* beliefs, int* labels) {
    const int pos = threadIdx.x & (G - 1);
    const int slot = (blockIdx.x * kBlock + threadIdx.x) / G;
    const Pixel px = map_slot(slot, a);
    if (!px.ok) return;
    const int x0 = pos * kLpl;
    const bool full = a.M == G * kLpl;
    PixelInputs in;
    load_pixel(a, px, x0, full, in);
    readout_pixel<G>(in, a.M, x0, full, beliefs ? beliefs + (size_t)px.p * a.M : nullptr,
                     labels ? labels + px.p : nullptr);
}

}  // namespace bpk
