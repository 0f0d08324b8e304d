// Sweep passes, max-product (Eq. 11 register / LDS window, Eq. 9 dense).
#include "bp_sweep_dispatch.hpp"

namespace bpk {

hipError_t launch_sweep_max(const UpdateArgs& a, bool dense, hipStream_t stream) {
    return dispatch_sweep<kMax>(a, dense, stream);
}

}  // namespace bpk
