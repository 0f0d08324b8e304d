// Sweep passes, sum-product (Eq. 7 register / LDS window, Eq. 2 dense).
#include "bp_sweep_dispatch.hpp"

namespace bpk {

hipError_t launch_sweep_max(const UpdateArgs& a, bool dense, hipStream_t stream);  // bp_launch_sweep_max.hip
hipError_t launch_sweep_sumf(const UpdateArgs& a, hipStream_t stream);              // bp_launch_sweep_sumf.hip

size_t sweep_dense_lds_need(int M, int mode) { return sweep_lds_bytes(lanes_for(M), M, mode, kSweepDense); }

hipError_t launch_sweep(const UpdateArgs& a, int mode, bool dense, hipStream_t stream) {
    const int len = (a.dir == kLeft || a.dir == kRight) ? a.W : a.H;
    if (len < 2) return hipSuccess;  // no sender has a neighbour this way
    if (mode == kSumF32) return dense ? hipErrorInvalidValue : launch_sweep_sumf(a, stream);
    return mode == kSum ? dispatch_sweep<kSum>(a, dense, stream) : launch_sweep_max(a, dense, stream);
}

}  // namespace bpk
