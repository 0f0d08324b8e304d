// Batched two-iteration max-product launches (Eq. 11): instantiations.
#include "bp_batch_pair_dispatch.hpp"

namespace bpk {

hipError_t launch_batch_pair_max(int arm, bool full, const BatchLaunch& L, unsigned grid, int parity,
                                 hipStream_t s) {
    return launch_batch_pair_arm<kMax>(arm, full, L, grid, parity, s);
}

}  // namespace bpk
