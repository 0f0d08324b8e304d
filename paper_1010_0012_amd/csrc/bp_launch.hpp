// Host-side launchers of the grid BP kernels (implemented in bp_launch_*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bp_device.hpp"

namespace bpk {

// Sparse O(mM) update of every message sent in one launch (a.colour < 0:
// all pixels; 0/1: one checkerboard colour).  mode: kSum / kMax.
hipError_t launch_sparse(const UpdateArgs& a, int mode, hipStream_t stream);
// Window half-width of the register variant launch_sparse would use for
// (M, T), or -1 for the runtime-window fallback.
int sparse_variant_tw(int M, int T);
// Two iterations in one launch, bitwise equal to two launch_sparse calls:
// synchronous (a.colour < 0: a.in -> a.out, the intermediate state into
// a.mid unless null), or a checkerboard pass pair (a.colour = c: the passes
// of colour 1 - c, then c, from a.in into the other buffer a.out == a.mid;
// the launch covers the colour-c slots).  sparse2_supported tells whether
// (M, T) has a compiled register window (otherwise run single launches).
bool sparse2_supported(int M, int T);
hipError_t launch_sparse2(const UpdateArgs& a, int mode, hipStream_t stream);
// Plain O(M^2) update, same contract (M <= 128); dense_lds_need gives the
// LDS bytes one workgroup needs.
size_t dense_lds_need(int M, int mode);
hipError_t launch_dense(const UpdateArgs& a, int mode, hipStream_t stream);
// One directional pass of the sweep schedule (a.dir = direction the messages
// travel, in place: a.in == a.out), sparse or dense; sweep_dense_lds_need
// gives the LDS bytes of the dense form (M <= 128).
hipError_t launch_sweep(const UpdateArgs& a, int mode, bool dense, hipStream_t stream);
size_t sweep_dense_lds_need(int M, int mode);
// General sparse-potential update (bp_launch_general.hip), same schedule
// contract as launch_sparse.
struct GenArgs;
hipError_t launch_general(const GenArgs& a, int mode, hipStream_t stream);
// One directional sweep pass with general potentials (a.u.dir, in place).
hipError_t launch_general_sweep(const GenArgs& a, int mode, hipStream_t stream);
// Factor-graph BP (bp_factor.hip): one synchronous iteration (variable ->
// factor, then factor -> variable), and the readout.
struct FgArgs;
// split: max-product with the split form (some f < fbar in C);
// most_entries: entries of the largest (type, slot) table (staged in LDS when
// it fits).
hipError_t launch_fg_iteration(const FgArgs& a, int mode, bool split, int most_entries, hipStream_t stream);
hipError_t launch_fg_beliefs(const FgArgs& a, float* beliefs, int* labels, hipStream_t stream);
// Batched two-iteration launch of one code path (bp_launch_batch_pair_*.hip);
// full: every instance of the launch has M = 4G.
struct BatchLaunch;
hipError_t launch_batch_pair_sum(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                 hipStream_t s);
hipError_t launch_batch_pair_max(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                 hipStream_t s);
// Sum-product in float32 arithmetic (full launches only).
hipError_t launch_batch_pair_sumf(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                  hipStream_t s);
// Dynamic LDS bytes for a launch whose kernel uses none, sized so that at
// most n of its workgroups fit in one CU's LDS (an occupancy cap) on the
// current device; 0 when the device cannot be queried.
size_t lds_cap_bytes(int n);
// Workgroups with `bytes` of dynamic LDS that fit in one CU of the current
// device (0 when they do not fit in a workgroup's LDS or the device cannot
// be queried).
int lds_blocks_per_cu(size_t bytes);
// Compute units of the current device (queried once per device); 0 when
// the device cannot be queried.
int cu_count();
// max |cur - prev| over the n (a multiple of 4) entries finite in both into
// *max_change, and the count of non-finite entries of cur into *non_finite
// (either output may be null; prev may be null: no change); both zeroed
// first on the stream.
hipError_t launch_message_stats(const float* cur, const float* prev, size_t n, float* max_change, int* non_finite,
                                hipStream_t s);
// Beliefs and/or MAP labels (either output may be null).
hipError_t launch_readout(const UpdateArgs& a, float* beliefs, int* labels, hipStream_t stream);
hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t stream);
// flag := 1 if some row of the [N][M] unary has a negative or non-finite
// entry or no positive entry, else 0.
hipError_t launch_validate_unary(const float* g, int N, int M, int* flag, hipStream_t stream);
// value into the inbox slots of off-grid neighbours of a [4][H][W][M] buffer
// (left slots of column 0, right of column W-1, up of row 0, down of row H-1).
hipError_t launch_fill_border(float* msg, int H, int W, int M, float value, hipStream_t stream);

}  // namespace bpk

namespace bpk {

struct AdjointArgs;
struct SeedArgs;
// Adjoint of synchronous sum-product BP (bp_launch_adjoint.hip).
bool adjoint_supported(int M, int T);
unsigned adjoint_blocks(int M, int N);  // workgroups of one adjoint launch
hipError_t launch_adjoint_seed(const SeedArgs& a, hipStream_t stream);
hipError_t launch_adjoint_step(const AdjointArgs& a, int T, hipStream_t stream);
hipError_t launch_sum_partials(const float* part, int n, float* out, hipStream_t stream);

}  // namespace bpk
