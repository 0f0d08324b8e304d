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
    // caller-owned device memory
    void* ws = nullptr;
    int64_t ws_bytes = 0;
    float* msg[2] = {nullptr, nullptr};  // synchronous ping-pong buffers
    int cur = 0;                          // buffer holding the current state
    int64_t cb_pass = 0;                  // checkerboard passes since reset
    const float* g = nullptr;

    size_t msg_floats() const { return (size_t)4 * N * M; }
};

namespace bpi {
int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
}  // namespace bpi
