// Host-side launchers of the grid BP kernels (implemented in bp_launch_*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bp_device.hpp"

namespace bpk {

// Labels per lane: the smallest power of two with 16 * LPL >= M.
inline int pick_lpl(int M) {
    int lpl = 1;
    while (kRow * lpl < M) lpl *= 2;
    return lpl;
}

// Neighbouring lanes each side the register window needs: ceil(T / LPL),
// at most the 15 other lanes of the row.
inline int window_lanes(int T, int lpl) {
    int k = (T + lpl - 1) / lpl;
    return k > kRow - 1 ? kRow - 1 : k;
}

// Sparse O(mM) update of every message sent in one launch (a.colour < 0:
// all pixels; 0/1: one checkerboard colour).  mode: kSum / kMax.
hipError_t launch_sparse(const UpdateArgs& a, int mode, hipStream_t stream);
// Which kernel launch_sparse would use: register window (K >= 0) or the
// runtime-window fallback (-1).
int sparse_variant_k(int M, int T);
// Plain O(M^2) update, same contract (M <= 128).
hipError_t launch_dense(const UpdateArgs& a, int mode, hipStream_t stream);
// Beliefs and/or MAP labels (either output may be null).
hipError_t launch_readout(const UpdateArgs& a, float* beliefs, int* labels, hipStream_t stream);
hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t stream);

}  // namespace bpk

namespace bpk {

struct AdjointArgs;
struct SeedArgs;
// Adjoint of synchronous sum-product BP (bp_launch_adjoint.hip).
bool adjoint_supported(int M, int T);
unsigned adjoint_blocks(int N);
hipError_t launch_adjoint_seed(const SeedArgs& a, hipStream_t stream);
hipError_t launch_adjoint_step(const AdjointArgs& a, int T, hipStream_t stream);
hipError_t launch_sum_partials(const float* part, int n, float* out, hipStream_t stream);

}  // namespace bpk
