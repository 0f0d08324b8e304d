// Sweep passes, sum-product in float32 arithmetic (Eq. 7, register windows).
#include "bp_sweep_dispatch.hpp"

namespace bpk {

hipError_t launch_sweep_sumf(const UpdateArgs& a, hipStream_t stream) {
    return dispatch_sweep<kSumF32>(a, false, stream);
}

}  // namespace bpk
