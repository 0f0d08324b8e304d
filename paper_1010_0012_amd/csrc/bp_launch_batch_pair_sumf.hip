// Batched two-iteration sum-product launches (Eq. 7) in float32 arithmetic:
// instantiations (full launches only).
#include "bp_batch_pair_dispatch.hpp"

namespace bpk {

hipError_t launch_batch_pair_sumf(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                  hipStream_t s) {
    return launch_batch_pair_arm<kSumF32>(arm, full, L, grid, parity, s);
}

}  // namespace bpk
