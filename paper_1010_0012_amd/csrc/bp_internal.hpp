// Host-side handle state of the grid BP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    const float* g = nullptr;
    // differentiation: set by bp_forward_ckpt, cleared by any state change
    bool grad_ready = false;
    int grad_n = 0, grad_k = 1;
    char* grad_ws = nullptr;

    size_t msg_floats() const { return (size_t)4 * N * M; }
};

// Workspace carving shared by the host files.
size_t bp_align_up(size_t v, size_t a);

namespace bpi {
int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int check_ready(const bp_grid* G);
int with_device(const bp_grid* G);
void invalidate_grad(bp_grid* G);
// Launch arguments for one update of G reading `in` and writing `out`
// (colour < 0: synchronous; 0/1: checkerboard pass of that colour).
bpk::UpdateArgs base_args(const bp_grid* G, const float* in, float* out, int colour);
}  // namespace bpi
