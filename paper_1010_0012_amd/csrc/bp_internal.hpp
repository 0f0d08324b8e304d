// Host-side handle state of the grid BP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "bp_device.hpp"

struct bp_grid {
    int dev = 0;
    hipStream_t stream = nullptr;
    int H = 0, W = 0, N = 0;
    // potential
    bool pot_set = false;
    int M = 0, T = 0;
    float alpha = 0.0f, fbar = 0.0f;
    bool fbar_tied = false;               // fbar = f(T), moves with alpha
    float tab_f[bpk::kMaxTab] = {};  // f(d), d <= T (0 beyond)
    float tab_w[bpk::kMaxTab] = {};  // f(d) - fbar, d <= T (0 beyond)
    double tab_wd[bpk::kDTab] = {};  // f(d) - fbar in double, d <= T (0 beyond)
    double fbar_d = 0.0;             // fbar in double (exact exp(-alpha T) when tied)
    // caller-owned device memory
    void* ws = nullptr;
    int64_t ws_bytes = 0;
    float* msg[2] = {nullptr, nullptr};  // synchronous ping-pong buffers
    int cur = 0;                          // buffer holding the current state
    int64_t cb_pass = 0;                  // checkerboard passes since reset
    bool fuse_sync = true;                // sync iterations run two per launch where compiled
    bool arith_f32 = false;               // BP_ARITH_F32: float32 arithmetic where compiled
    int pair_layout = bpk::kPairWide;     // two-iteration launch mapping (bpk::PairLayout)
    bool pair_layout_set = false;         // chosen by bp_set_launch_tuning or bp_autotune (else it follows the arithmetic)
    int pair_cap = -1;                    // its workgroups per CU (0: no cap, -1: the default)
    const float* g = nullptr;
    // general sparse potentials (bp_set_sparse_potentials), or the Eq. 10
    // tables of the window potential built into the workspace's table region
    bool general = false;                 // bp_iterate runs the general kernel on the caller's tables
    int gen_types = 0, gen_top_k = 0, gen_mask_words = 0;
    int gen_entries = 0;                  // table entries of both orientations
    float gen_fbar[16] = {};
    double gen_fbar_d[16] = {};
    int gen_eq10[16] = {};
    char* gen_tab = nullptr;              // device tables
    size_t gen_off[5] = {};               // offsets of ptr, ent_x, ent_f, ent_w, mask
    const uint8_t* type_h = nullptr;      // borrowed edge-type maps (null: type 0)
    const uint8_t* type_v = nullptr;
    std::vector<char> gen_host;           // host image of the tables (the upload's source)
    bool win_tab_valid = false;           // window tables in the workspace match (T, alpha, fbar)
    // differentiation: set by bp_forward_ckpt, cleared by any state change
    bool grad_ready = false;
    int grad_n = 0, grad_k = 1;
    char* grad_ws = nullptr;

    size_t msg_floats() const { return (size_t)4 * N * M; }
};

// BP_DEBUG builds check the host side's workspace carving and index
// arithmetic as they go and abort on the first violation (host code only;
// the sanitizer build of the host runtime compiles with it).
#ifdef BP_DEBUG
#include <cstdio>
#include <cstdlib>
#define BP_ASSERT(cond)                                                                     \
    do {                                                                                    \
        if (!(cond)) {                                                                      \
            std::fprintf(stderr, "BP_ASSERT failed: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
            std::abort();                                                                   \
        }                                                                                   \
    } while (0)
#else
#define BP_ASSERT(cond) ((void)0)
#endif

// Workspace carving shared by the host files.
size_t bp_align_up(size_t v, size_t a);

namespace bpi {
int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int check_ready(const bp_grid* G);
int with_device(const bp_grid* G);
void invalidate_grad(bp_grid* G);
// True when the float32 window table has f(d) >= fbar for every |d| <= T
// (Eq. 11 holds for max-product; otherwise Eq. 10 is needed).
bool max_product_ok(const bp_grid* G);
// Launch arguments for one update of G reading `in` and writing `out`
// (colour < 0: synchronous; 0/1: checkerboard pass of that colour).
bpk::UpdateArgs base_args(const bp_grid* G, const float* in, float* out, int colour);
// Device bytes of the window-potential table region at the end of the
// workspace (Eq. 10 fallback of max-product when fbar exceeds f).
size_t window_table_bytes(int M);
// Byte offset in the workspace of the int flag of the unary check (after the
// two message buffers and the window tables).
inline size_t validate_flag_offset(const bp_grid* G) {
    return 2 * bp_align_up(G->msg_floats() * sizeof(float), 256) + bp_align_up(window_table_bytes(G->M), 256);
}
// n iterations through the general kernel (caller's tables, or the window
// potential's Eq. 10 tables); schedule sync, checkerboard or sweep.
int iterate_general(bp_grid* G, int kmode, int n, int schedule);
// One launch of the general kernel with G's tables over the grid, buffers
// and schedule that u describes (a level of the multi-scale pyramid).
hipError_t launch_general_update(const bp_grid* G, const bpk::UpdateArgs& u, int kmode);
// Build the window potential's tables into the workspace table region.
int build_window_tables(bp_grid* G);
// A named roctx range for the life of the object, for rocprofv3
// --marker-trace, when the process runs with BP_ROCTX=1; roctx is looked up
// at run time (dlopen), so the library does not depend on it, and without
// the variable (or without roctx) the range costs one branch.
struct TraceRange {
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
    bool on;
};
}  // namespace bpi
