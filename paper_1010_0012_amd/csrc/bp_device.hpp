// Device-side building blocks shared by every BP kernel (gfx950, wave64).
//
// Mapping: one pixel per 16-lane DPP row.  Lane l of the row owns the LPL
// consecutive labels [l*LPL, (l+1)*LPL); the row's capacity is 16*LPL >= M
// and labels >= M are padding that holds h = 0.  Cross-lane traffic stays
// inside a row, so every row-wide reduction and every label shift is a DPP
// modifier on an ordinary VALU op: no LDS, no barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpk {

constexpr int kRow = 16;            // lanes per pixel (one DPP row)
#ifndef BP_BLOCK
#define BP_BLOCK 256
#endif
constexpr int kBlock = BP_BLOCK;    // threads per workgroup (16 lanes per pixel row)
constexpr int kMaxTab = 256;        // potential table entries (|d| < BP_MAX_LABELS)

enum Mode { kSum = 0, kMax = 1 };

#ifndef BP_MSG_NT
#define BP_MSG_NT 1
#endif
#ifndef BP_UNARY_NT
#define BP_UNARY_NT 1
#endif
constexpr bool kMsgNT = BP_MSG_NT;      // message loads/stores non-temporal
constexpr bool kUnaryNT = BP_UNARY_NT;  // unary loads non-temporal

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
    float fbar;            // potential outside the window
    float tab[kMaxTab];    // sum: f(d) - fbar for d <= T, 0 beyond; max/dense: f(d) for d <= T
};

// ---------------------------------------------------------------- DPP ----
// DPP16 controls (GFX9 encoding).
constexpr int kQuad1032 = 0xB1;     // quad_perm:[1,0,3,2]
constexpr int kQuad2301 = 0x4E;     // quad_perm:[2,3,0,1]
constexpr int kRowMirror = 0x140;   // lane i <- lane 15-i
constexpr int kRowHalfMirror = 0x141; // lane i <- lane 7-i within each half row
constexpr int row_shl(int j) { return 0x100 + j; }  // lane i <- lane i+j (0 past the row end)
constexpr int row_shr(int j) { return 0x110 + j; }  // lane i <- lane i-j (0 before the row start)

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    // old = 0 and bound_ctrl: lanes whose source lies outside the row read 0.
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// Butterfly over the 16 lanes of a row; every lane ends with the same bits
// (each step adds two operands that are the same pair on both partners).
__device__ __forceinline__ float row_sum(float v) {
    v += dpp<kQuad1032>(v);
    v += dpp<kQuad2301>(v);
    v += dpp<kRowHalfMirror>(v);
    v += dpp<kRowMirror>(v);
    return v;
}

__device__ __forceinline__ float row_max(float v) {
    v = fmaxf(v, dpp<kQuad1032>(v));
    v = fmaxf(v, dpp<kQuad2301>(v));
    v = fmaxf(v, dpp<kRowHalfMirror>(v));
    v = fmaxf(v, dpp<kRowMirror>(v));
    return v;
}

template <int MODE>
__device__ __forceinline__ float row_reduce(float v) {
    if constexpr (MODE == kSum) return row_sum(v); else return row_max(v);
}

// ------------------------------------------------------- label vectors ----
typedef float v2f __attribute__((ext_vector_type(2)));
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

// Load this lane's LPL labels of one pixel row (base points at label 0).
// full: M == 16*LPL, so the lane's labels are all real and 4*LPL-byte
// aligned; otherwise labels >= M read `fill`.
template <int LPL, bool NT>
__device__ __forceinline__ void load_labels(const float* base, int x0, int M, bool full,
                                            float (&v)[LPL], float fill) {
    if (full) {
        if constexpr (LPL == 1) {
            v[0] = ld(base + x0, NT);
        } else if constexpr (LPL == 2) {
            v2f t = ld(reinterpret_cast<const v2f*>(base + x0), NT);
            v[0] = t.x; v[1] = t.y;
        } else {
#pragma unroll
            for (int i = 0; i < LPL; i += 4) {
                v4f t = ld(reinterpret_cast<const v4f*>(base + x0 + i), NT);
                v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < LPL; ++i) v[i] = (x0 + i < M) ? ld(base + x0 + i, NT) : fill;
    }
}

template <int LPL, bool NT>
__device__ __forceinline__ void store_labels(float* base, int x0, int M, bool full,
                                             const float (&v)[LPL]) {
    if (full) {
        if constexpr (LPL == 1) {
            st(base + x0, v[0], NT);
        } else if constexpr (LPL == 2) {
            st(reinterpret_cast<v2f*>(base + x0), v2f{v[0], v[1]}, NT);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; i += 4)
                st(reinterpret_cast<v4f*>(base + x0 + i), v4f{v[i], v[i + 1], v[i + 2], v[i + 3]}, NT);
        }
    } else {
#pragma unroll
        for (int i = 0; i < LPL; ++i)
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
template <int LPL>
struct PixelInputs {
    float g[LPL];
    float m[4][LPL];
};

// Load the unary and the inbox of one pixel from explicit pointers (plane =
// N*M floats between inbox planes); off-grid neighbours read as 1.
template <int LPL>
__device__ __forceinline__ void load_pixel_ptr(const float* g, const float* in, size_t plane, int M,
                                               const Pixel& px, int x0, bool full,
                                               PixelInputs<LPL>& r) {
    const size_t off = (size_t)px.p * M;
    load_labels<LPL, kUnaryNT>(g + off, x0, M, full, r.g, 0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (px.has[k]) {
            load_labels<LPL, kMsgNT>(in + k * plane + off, x0, M, full, r.m[k], 1.0f);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) r.m[k][i] = 1.0f;
        }
    }
}

template <int LPL>
__device__ __forceinline__ void load_pixel(const UpdateArgs& a, const Pixel& px, int x0, bool full,
                                           PixelInputs<LPL>& in) {
    load_pixel_ptr<LPL>(a.g, a.in, (size_t)a.N * a.M, a.M, px, x0, full, in);
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

// Eq. 5 for the four outgoing messages: h_o = g * product of the inbox
// messages except the one from the target o.  Shared partial products:
// gUD = g*mU*mD serves the horizontal targets, gLR = g*mL*mR the vertical
// ones (8 multiplies per label for the four vectors).  Padding labels have
// g = 0, hence h = 0.
template <int LPL>
__device__ __forceinline__ void make_h(const PixelInputs<LPL>& in, float (&h)[4][LPL]) {
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        const float gud = (in.g[i] * in.m[kUp][i]) * in.m[kDown][i];
        const float glr = (in.g[i] * in.m[kLeft][i]) * in.m[kRight][i];
        h[kLeft][i] = gud * in.m[kRight][i];   // to the left neighbour: skip its message
        h[kRight][i] = gud * in.m[kLeft][i];
        h[kUp][i] = glr * in.m[kDown][i];
        h[kDown][i] = glr * in.m[kUp][i];
    }
}

// Normalise u (Sec. 3: explicit normalisation after each update) with one
// IEEE division per message, then store into the receiver's inbox slot.
template <int LPL>
__device__ __forceinline__ void normalise_store_ptr(float* out, size_t plane, int M, int W,
                                                    const Pixel& px, int dir, int x0, bool full,
                                                    float (&u)[LPL]) {
    float z = 0.0f;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
        if (!full && x0 + i >= M) u[i] = 0.0f;
        z += u[i];
    }
    z = row_sum(z);
    const float inv = 1.0f / z;
#pragma unroll
    for (int i = 0; i < LPL; ++i) u[i] *= inv;
    if (px.ok && px.has[dir]) {
        const int q = neighbour(px, dir, W);
        store_labels<LPL, kMsgNT>(out + opposite(dir) * plane + (size_t)q * M, x0, M, full, u);
    }
}

template <int LPL>
__device__ __forceinline__ void normalise_store(const UpdateArgs& a, const Pixel& px, int dir,
                                                int x0, bool full, float (&u)[LPL]) {
    normalise_store_ptr<LPL>(a.out, (size_t)a.N * a.M, a.M, a.W, px, dir, x0, full, u);
}

}  // namespace bpk
