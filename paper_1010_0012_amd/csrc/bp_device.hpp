// Device-side building blocks shared by every BP kernel (gfx950, wave64).
//
// Mapping: one pixel per group of G lanes, G = 4, 8, 16, 32 or 64, each lane
// owning kLpl = 4 consecutive labels [4*pos, 4*pos + 4) with pos = lane mod G:
// the group holds 4*G >= M labels and labels >= M are padding with h = 0.
// Every label row is therefore read and written as one float4 per lane, and
// a wave's load or store instruction covers 64/G consecutive pixels'
// contiguous rows.  (With 8 labels per lane, two float4 per lane at a 32-byte
// lane stride, the same memory pattern measured 4.75 TB/s on MI355X against
// 6.0 TB/s for one float4 per lane at M = 128.)
//
// Cross-lane traffic stays inside the group: reductions are DPP butterflies
// (quad_perm, row_half_mirror, row_mirror) plus, for G >= 32, ds_swizzle
// (xor 16) and ds_bpermute (xor 32); label shifts are DPP row_shr/row_shl
// (G <= 16) or chained wave_shr/wave_shl by one lane (G >= 32), with the
// lanes that would read another pixel's labels zeroed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpk {

constexpr int kLpl = 4;             // labels per lane
#ifndef BP_BLOCK
#define BP_BLOCK 256
#endif
constexpr int kBlock = BP_BLOCK;    // threads per workgroup
constexpr int kMaxTab = 256;        // potential table entries (|d| < BP_MAX_LABELS)
constexpr int kDTab = 32;           // double window weights carried in the arguments (|d| <= 31)

// Mappings of the two-iteration launch (UpdateArgs::pair_layout).
enum PairLayout { kPairStrips = 0, kPairBands = 1, kPairSlots = 2, kPairWide = 3, kPairWalk = 4, kPairTile = 5 };

// kSumF32: sum-product with float32 arithmetic (BP_ARITH_F32), used by the
// synchronous and checkerboard window kernels only.
enum Mode { kSum = 0, kMax = 1, kSumF32 = 2 };

#ifndef BP_MSG_NT
#define BP_MSG_NT 1
#endif
#ifndef BP_UNARY_NT
#define BP_UNARY_NT 1
#endif
constexpr bool kMsgNT = BP_MSG_NT;      // message loads/stores non-temporal
constexpr bool kUnaryNT = BP_UNARY_NT;  // unary loads non-temporal

// Lanes per pixel for M labels: the smallest power of two >= ceil(M/4), at
// least 4 (a quad) and at most 64 (a wave).
constexpr int lanes_for(int M) {
    int g = 4;
    while (g * kLpl < M && g < 64) g *= 2;
    return g;
}

// Inbox directions: where the sender sits relative to the receiver.
enum Dir { kLeft = 0, kRight = 1, kUp = 2, kDown = 3 };

// Arguments of one grid-wide update launch.  Passed by value: the table
// lands in the kernarg segment and taps with compile-time indices become
// scalar loads.
struct UpdateArgs {
    const float* g;        // unary [N][M]
    const float* in;       // inbox planes read  [4][N][M]
    float* out;            // inbox planes written [4][N][M] (== in for checkerboard)
    int H, W, M, N;
    int colour;            // -1: every pixel sends; 0/1: only (r + c) % 2 == colour
    int half_w;            // (W + 1) / 2, checkerboard slot mapping
    int n_slots;           // pixels (or checkerboard slots) covered by the launch
    int T;                 // truncation (used by the runtime-window kernels)
    int dir;               // sweep pass: direction the messages travel (kLeft .. kDown)
    int both;              // sweep: 1 = the second half of the grid runs the opposite direction
    int eq10;              // max-product: some f(d) < fbar, so Eq. 10 (not Eq. 11) holds
    float* mid;            // two-iteration launches: where the first iteration's messages go, or null
    int pair_layout;       // two-iteration launch mapping (host side, PairLayout): row blocks in XCD
                           // column strips, in XCD row bands or in one wide strip per XCD; one group per slot
    int pair_cap;          // workgroups per CU allowed by the launch's LDS request: 0 none, -1 the default
    float fbar;            // potential outside the window (float32, max-product)
    float tab[kMaxTab];    // max-product: f(d) for d <= T, 0 beyond (float32)
    // Sum-product works in double end to end: the potential in double and
    // every accumulation in double, messages rounded once to float32.
    double fbar_d;         // fbar in double
    double alpha_d;        // alpha in double (tables built on the device)
    double dtab[kDTab];    // f(d) - fbar in double for d <= min(T, kDTab-1), 0 beyond T
};

// ---------------------------------------------------------------- DPP ----
// DPP16 controls (GFX9 encoding).
constexpr int kQuad1032 = 0xB1;       // quad_perm:[1,0,3,2]
constexpr int kQuad2301 = 0x4E;       // quad_perm:[2,3,0,1]
constexpr int kRowMirror = 0x140;     // lane i <- lane 15-i
constexpr int kRowHalfMirror = 0x141; // lane i <- lane 7-i within each half row
constexpr int kWaveShl1 = 0x130;      // lane i <- lane i+1 across the wave
constexpr int kWaveShr1 = 0x138;      // lane i <- lane i-1 across the wave
constexpr int row_shl(int j) { return 0x100 + j; }  // lane i <- lane i+j (0 past the row end)
constexpr int row_shr(int j) { return 0x110 + j; }  // lane i <- lane i-j (0 before the row start)
constexpr int kSwizzleXor16 = 0x401F; // ds_swizzle bit mode: lane i <- lane i^16 (within 32)

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    // old = 0 and bound_ctrl: lanes whose source lies outside the row read 0.
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ float xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), kSwizzleXor16));
}
__device__ __forceinline__ int xor16_i(int v) { return __builtin_amdgcn_ds_swizzle(v, kSwizzleXor16); }
__device__ __forceinline__ float xor32(float v) {
    const int src = ((int)(threadIdx.x & 63) ^ 32) << 2;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}
__device__ __forceinline__ int xor32_i(int v) {
    const int src = ((int)(threadIdx.x & 63) ^ 32) << 2;
    return __builtin_amdgcn_ds_bpermute(src, v);
}

// Butterfly over the G lanes of a pixel; every lane ends with the same bits
// (each step adds two operands that are the same pair on both partners).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    v += dpp<kQuad1032>(v);
    v += dpp<kQuad2301>(v);
    if constexpr (G >= 8) v += dpp<kRowHalfMirror>(v);
    if constexpr (G >= 16) v += dpp<kRowMirror>(v);
    if constexpr (G >= 32) v += xor16(v);
    if constexpr (G >= 64) v += xor32(v);
    return v;
}

template <int G>
__device__ __forceinline__ float group_max(float v) {
    v = fmaxf(v, dpp<kQuad1032>(v));
    v = fmaxf(v, dpp<kQuad2301>(v));
    if constexpr (G >= 8) v = fmaxf(v, dpp<kRowHalfMirror>(v));
    if constexpr (G >= 16) v = fmaxf(v, dpp<kRowMirror>(v));
    if constexpr (G >= 32) v = fmaxf(v, xor16(v));
    if constexpr (G >= 64) v = fmaxf(v, xor32(v));
    return v;
}

template <int MODE, int G>
__device__ __forceinline__ float group_reduce(float v) {
    if constexpr (MODE == kSum) return group_sum<G>(v); else return group_max<G>(v);
}

// Double-precision shuffles: each 32-bit half moves with the same pattern.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double xor16_d(double v) {
    return __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(v), kSwizzleXor16),
                            __builtin_amdgcn_ds_swizzle(__double2loint(v), kSwizzleXor16));
}
__device__ __forceinline__ double xor32_d(double v) {
    const int src = ((int)(threadIdx.x & 63) ^ 32) << 2;
    return __hiloint2double(__builtin_amdgcn_ds_bpermute(src, __double2hiint(v)),
                            __builtin_amdgcn_ds_bpermute(src, __double2loint(v)));
}

// The two rows of an xor-16 (or xor-32) lane pair, on the VALU: with
// both operands v, v_permlane16_swap leaves lane i with the values of lanes
// i & ~16 and i | 16 (v_permlane32_swap: i & ~32 and i | 32), the same pair
// in the same order on both partners.
__device__ __forceinline__ void rows16_d(double v, double& lo_row, double& hi_row) {
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false,
                                                    false);
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false,
                                                    false);
    lo_row = __hiloint2double((int)h[0], (int)l[0]);
    hi_row = __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ void rows32_d(double v, double& lo_half, double& hi_half) {
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false,
                                                    false);
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false,
                                                    false);
    lo_half = __hiloint2double((int)h[0], (int)l[0]);
    hi_half = __hiloint2double((int)h[1], (int)l[1]);
}

// Group sum in double (the sum-product accumulations; same butterfly, so
// every lane ends with the same bits).  The steps across rows add the pair
// from the row swaps: the same two operands as lane + partner, so the same
// bits, without a trip through the LDS pipe.
template <int G>
__device__ __forceinline__ double group_sum_d(double v) {
    v += dpp_d<kQuad1032>(v);
    v += dpp_d<kQuad2301>(v);
    if constexpr (G >= 8) v += dpp_d<kRowHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_d<kRowMirror>(v);
    double a, b;
    if constexpr (G >= 32) {
        rows16_d(v, a, b);
        v = a + b;
    }
    if constexpr (G >= 64) {
        rows32_d(v, a, b);
        v = a + b;
    }
    return v;
}

template <int G>
__device__ __forceinline__ double group_max_d(double v) {
    v = fmax(v, dpp_d<kQuad1032>(v));
    v = fmax(v, dpp_d<kQuad2301>(v));
    if constexpr (G >= 8) v = fmax(v, dpp_d<kRowHalfMirror>(v));
    if constexpr (G >= 16) v = fmax(v, dpp_d<kRowMirror>(v));
    double a, b;
    if constexpr (G >= 32) {
        rows16_d(v, a, b);
        v = fmax(a, b);
    }
    if constexpr (G >= 64) {
        rows32_d(v, a, b);
        v = fmax(a, b);
    }
    return v;
}

// (value, index) tournament over the group: larger value wins, the lower
// index breaks ties; the result is the same on every lane.
template <int G>
__device__ __forceinline__ void group_argmax(float& best, int& arg) {
    auto take = [&](float ob, int oa) {
        if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
    };
    take(dpp<kQuad1032>(best), dpp_i<kQuad1032>(arg));
    take(dpp<kQuad2301>(best), dpp_i<kQuad2301>(arg));
    if constexpr (G >= 8) take(dpp<kRowHalfMirror>(best), dpp_i<kRowHalfMirror>(arg));
    if constexpr (G >= 16) take(dpp<kRowMirror>(best), dpp_i<kRowMirror>(arg));
    if constexpr (G >= 32) take(xor16(best), xor16_i(arg));
    if constexpr (G >= 64) take(xor32(best), xor32_i(arg));
}

// (value, label) tournament in double: larger value wins, the lower label
// breaks ties; the same result on every lane of the group.
template <int G>
__device__ __forceinline__ void group_argmax_d(double& best, int& arg) {
    auto take = [&](double ob, int oa) {
        if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
    };
    take(dpp_d<kQuad1032>(best), dpp_i<kQuad1032>(arg));
    take(dpp_d<kQuad2301>(best), dpp_i<kQuad2301>(arg));
    if constexpr (G >= 8) take(dpp_d<kRowHalfMirror>(best), dpp_i<kRowHalfMirror>(arg));
    if constexpr (G >= 16) take(dpp_d<kRowMirror>(best), dpp_i<kRowMirror>(arg));
    if constexpr (G >= 32) take(xor16_d(best), xor16_i(arg));
    if constexpr (G >= 64) take(xor32_d(best), xor32_i(arg));
}

// Slot of label x in a group's LDS row of G*4 doubles: (x mod 4) * G + x / 4.
// Lane pos owns labels 4*pos .. 4*pos+3, so its own writes (label 4*pos + i
// at i*G + pos) and reads at a fixed offset from its labels fall on
// consecutive doubles across the group's lanes: no bank conflicts, where the
// plain label index (a 32-byte stride between lanes) hits a quarter of the
// banks.
template <int G>
__device__ __forceinline__ int row_slot(int x) { return (x & (kLpl - 1)) * G + (x >> 2); }

// Order this wave's LDS accesses: writes before the call are visible to
// every lane of the wave after it.  Enough wherever only the lanes of one
// G-lane group (G <= 64, so inside one wave) share an LDS row.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The k largest entries of the group's label vector (this lane holds labels
// x0 .. x0+3 of v, labels >= M ignored), value descending and label
// ascending on ties; lane 0 of the group writes them to top_v / top_i.  k
// rounds of the tournament, each taking the best entry after the previous.
template <int G>
__device__ __forceinline__ void group_top_k(const double (&v)[kLpl], int M, int x0, int pos, int k, double* top_v,
                                            int* top_i) {
    double last_v = __builtin_huge_val();
    int last_i = -1;
    for (int r = 0; r < k; ++r) {
        double bv = -1.0;
        int bi = 1 << 30;
#pragma unroll
        for (int i = 0; i < kLpl; ++i) {
            const int y = x0 + i;
            const bool after = v[i] < last_v || (v[i] == last_v && y > last_i);
            if (y < M && after && (v[i] > bv || (v[i] == bv && y < bi))) { bv = v[i]; bi = y; }
        }
        group_argmax_d<G>(bv, bi);
        if (pos == 0) { top_v[r] = bv; top_i[r] = bi; }
        last_v = bv;
        last_i = bi;
    }
}

// Label shifts inside the group: lane pos receives lane pos-J (from_lower)
// or pos+J (from_upper) of the same pixel, 0 where that lane does not exist.
template <int G, int J>
__device__ __forceinline__ float from_lower(float v, int pos) {
    static_assert(G <= 16, "wide groups shift one lane at a time");
    const float t = dpp<row_shr(J)>(v);
    if constexpr (G == 16) return t;
    else return pos < J ? 0.0f : t;
}
template <int G, int J>
__device__ __forceinline__ float from_upper(float v, int pos) {
    static_assert(G <= 16, "wide groups shift one lane at a time");
    const float t = dpp<row_shl(J)>(v);
    if constexpr (G == 16) return t;
    else return pos >= G - J ? 0.0f : t;
}
template <int G>
__device__ __forceinline__ float lower1(float v, int pos) {  // G >= 32: one lane across rows
    const float t = dpp<kWaveShr1>(v);
    return pos == 0 ? 0.0f : t;
}
template <int G>
__device__ __forceinline__ float upper1(float v, int pos) {
    const float t = dpp<kWaveShl1>(v);
    return pos == G - 1 ? 0.0f : t;
}

// The same shifts for doubles (both halves move together).
template <int G, int J>
__device__ __forceinline__ double from_lower_d(double v, int pos) {
    static_assert(G <= 16, "wide groups shift one lane at a time");
    const double t = dpp_d<row_shr(J)>(v);
    if constexpr (G == 16) return t;
    else return pos < J ? 0.0 : t;
}
template <int G, int J>
__device__ __forceinline__ double from_upper_d(double v, int pos) {
    static_assert(G <= 16, "wide groups shift one lane at a time");
    const double t = dpp_d<row_shl(J)>(v);
    if constexpr (G == 16) return t;
    else return pos >= G - J ? 0.0 : t;
}
template <int G>
__device__ __forceinline__ double lower1_d(double v, int pos) {
    const double t = dpp_d<kWaveShr1>(v);
    return pos == 0 ? 0.0 : t;
}
template <int G>
__device__ __forceinline__ double upper1_d(double v, int pos) {
    const double t = dpp_d<kWaveShl1>(v);
    return pos == G - 1 ? 0.0 : t;
}

// ------------------------------------------------------- label vectors ----
typedef float v4f __attribute__((ext_vector_type(4)));

// Streaming hint: every message and unary entry is touched once per launch
// and a large grid's working set is far beyond the caches, so the update
// loads and stores non-temporally (measured on 480x640, M=64: 114.7 us per
// launch against 125.0 us with the default policy).
template <typename T>
__device__ __forceinline__ T ld(const T* p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}
template <typename T>
__device__ __forceinline__ void st(T* p, T v, bool nt) {
    if (nt) __builtin_nontemporal_store(v, p); else *p = v;
}

// Load this lane's 4 labels of one pixel row (base points at label 0).
// full: M == 4*G, so every lane's float4 is real and 16-byte aligned;
// otherwise labels >= M read `fill` (and M need not be a multiple of 4).
template <bool NT>
__device__ __forceinline__ void load_labels(const float* base, int x0, int M, bool full,
                                            float (&v)[kLpl], float fill) {
    if (full) {
        const v4f t = ld(reinterpret_cast<const v4f*>(base + x0), NT);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
#pragma unroll
        for (int i = 0; i < kLpl; ++i) v[i] = (x0 + i < M) ? ld(base + x0 + i, NT) : fill;
    }
}

template <bool NT>
__device__ __forceinline__ void store_labels(float* base, int x0, int M, bool full,
                                             const float (&v)[kLpl]) {
    if (full) {
        st(reinterpret_cast<v4f*>(base + x0), v4f{v[0], v[1], v[2], v[3]}, NT);
    } else {
#pragma unroll
        for (int i = 0; i < kLpl; ++i)
            if (x0 + i < M) st(base + x0 + i, v[i], NT);
    }
}

// ------------------------------------------------------- pixel mapping ----
struct Pixel {
    int r, c, p;
    bool ok;
    bool has[4];
};

// Slot -> pixel.  Synchronous launches cover every pixel row-major; a
// checkerboard pass covers H * ceil(W/2) slots, the j-th slot of row r being
// column 2j + ((colour + r) & 1), which is off the grid for some odd-W rows.
__device__ __forceinline__ Pixel map_slot(int slot, const UpdateArgs& a) {
    Pixel px;
    if (a.colour < 0) {
        px.r = slot / a.W;
        px.c = slot - px.r * a.W;
    } else {
        px.r = slot / a.half_w;
        int j = slot - px.r * a.half_w;
        px.c = 2 * j + ((a.colour + px.r) & 1);
    }
    px.ok = slot < a.n_slots && px.c < a.W;
    px.p = px.r * a.W + px.c;
    px.has[kLeft] = px.c > 0;
    px.has[kRight] = px.c + 1 < a.W;
    px.has[kUp] = px.r > 0;
    px.has[kDown] = px.r + 1 < a.H;
    return px;
}

// Synchronous slot -> pixel (row-major).
__device__ __forceinline__ Pixel sync_pixel(int slot, int H, int W, int N) {
    Pixel px;
    px.r = slot / W;
    px.c = slot - px.r * W;
    px.ok = slot < N;
    px.p = px.r * W + px.c;
    px.has[kLeft] = px.c > 0;
    px.has[kRight] = px.c + 1 < W;
    px.has[kUp] = px.r > 0;
    px.has[kDown] = px.r + 1 < H;
    return px;
}

__device__ __forceinline__ int neighbour(const Pixel& px, int dir, int W) {
    switch (dir) {
        case kLeft: return px.p - 1;
        case kRight: return px.p + 1;
        case kUp: return px.p - W;
        default: return px.p + W;
    }
}

__device__ __forceinline__ constexpr int opposite(int dir) { return dir ^ 1; }

// The unary and the four inbox messages of one pixel (this lane's labels).
struct PixelInputs {
    float g[kLpl];
    float m[4][kLpl];
};

// Inputs of a slot that maps to no pixel: finite values whose results are
// never stored.
__device__ __forceinline__ void dummy_pixel(PixelInputs& r) {
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        r.g[i] = 1.0f;
        r.m[0][i] = r.m[1][i] = r.m[2][i] = r.m[3][i] = 1.0f;
    }
}

// Load the unary and the inbox of one pixel from explicit pointers (plane =
// N*M floats between inbox planes); off-grid neighbours read as 1.
__device__ __forceinline__ void load_pixel_ptr(const float* g, const float* in, size_t plane, int M,
                                               const Pixel& px, int x0, bool full, PixelInputs& r) {
    const size_t off = (size_t)px.p * M;
    load_labels<kUnaryNT>(g + off, x0, M, full, r.g, 0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (px.has[k]) {
            load_labels<kMsgNT>(in + k * plane + off, x0, M, full, r.m[k], 1.0f);
        } else {
#pragma unroll
            for (int i = 0; i < kLpl; ++i) r.m[k][i] = 1.0f;
        }
    }
}

__device__ __forceinline__ void load_pixel(const UpdateArgs& a, const Pixel& px, int x0, bool full,
                                           PixelInputs& in) {
    load_pixel_ptr(a.g, a.in, (size_t)a.N * a.M, a.M, px, x0, full, in);
}

// Eq. 5 for the four outgoing messages: h_o = g * product of the inbox
// messages except the one from the target o.  Shared partial products:
// gUD = g*mU*mD serves the horizontal targets, gLR = g*mL*mR the vertical
// ones (8 multiplies per label for the four vectors).  Padding labels have
// g = 0, hence h = 0.
__device__ __forceinline__ void make_h(const PixelInputs& in, float (&h)[4][kLpl]) {
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        const float gud = (in.g[i] * in.m[kUp][i]) * in.m[kDown][i];
        const float glr = (in.g[i] * in.m[kLeft][i]) * in.m[kRight][i];
        h[kLeft][i] = gud * in.m[kRight][i];   // to the left neighbour: skip its message
        h[kRight][i] = gud * in.m[kLeft][i];
        h[kUp][i] = glr * in.m[kDown][i];
        h[kDown][i] = glr * in.m[kUp][i];
    }
}

// make_h in double (the max-product path): g * m is exact in double, so h
// carries at most two double roundings and every max-product message is its
// exact value rounded once to float32 at the store.
__device__ __forceinline__ void make_h_d(const PixelInputs& in, double (&h)[4][kLpl]) {
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        const double g = in.g[i];
        const double gud = (g * in.m[kUp][i]) * in.m[kDown][i];
        const double glr = (g * in.m[kLeft][i]) * in.m[kRight][i];
        h[kLeft][i] = gud * in.m[kRight][i];
        h[kRight][i] = gud * in.m[kLeft][i];
        h[kUp][i] = glr * in.m[kDown][i];
        h[kDown][i] = glr * in.m[kUp][i];
    }
}

// Store a finished message into the receiver's inbox slot.
__device__ __forceinline__ void store_message(float* out, size_t plane, int M, int W, const Pixel& px,
                                              int dir, int x0, bool full, const float (&m)[kLpl]) {
    if (px.ok && px.has[dir]) {
        const int q = neighbour(px, dir, W);
        store_labels<kMsgNT>(out + opposite(dir) * plane + (size_t)q * M, x0, M, full, m);
    }
}

// 1/z in double from the hardware reciprocal and two Newton steps (each
// roughly doubles the correct bits), ample for a result rounded to float.
__device__ __forceinline__ double recip_d(double z) {
    double r = __builtin_amdgcn_rcp(z);
    r = fma(r, fma(-z, r, 1.0), r);
    r = fma(r, fma(-z, r, 1.0), r);
    return r;
}

// Normalisation (Sec. 3) in double, both modes: Z = sum of u over the
// group, one reciprocal per message, m = u / Z rounded once to float.
template <int G>
__device__ __forceinline__ void normalise_d(double (&u)[kLpl], int M, int x0, bool full, float (&m)[kLpl]) {
    double z = 0.0;
#pragma unroll
    for (int i = 0; i < kLpl; ++i) {
        if (!full && x0 + i >= M) u[i] = 0.0;
        z += u[i];
    }
    z = group_sum_d<G>(z);
    const double inv = recip_d(z);
#pragma unroll
    for (int i = 0; i < kLpl; ++i) m[i] = (float)(u[i] * inv);
}

// Eq. 3 for this lane's labels: the product of the unary and the four
// incoming messages formed in double (five float32 factors: no underflow,
// whose smallest product is about 1e-224, and at most three roundings), then
// normalised in double and rounded once to float32, as every message is.
// Only a row whose product is exactly zero for every label (a unary row with
// no positive entry, which bp_set_unary's contract excludes) gives 0/0.
template <int G>
__device__ __forceinline__ void belief_d(const PixelInputs& in, int M, int x0, bool full, float (&b)[kLpl]) {
    double p[kLpl];
#pragma unroll
    for (int i = 0; i < kLpl; ++i)
        p[i] = ((((double)in.g[i] * in.m[kLeft][i]) * in.m[kRight][i]) * in.m[kUp][i]) * in.m[kDown][i];
    normalise_d<G>(p, M, x0, full, b);
}

}  // namespace bpk
