// Sparse O(mM) sum-product update (Eq. 7) in float32 arithmetic:
// instantiations and dispatch (register windows; pairs as row-block launches).
#include "bp_sparse_dispatch.hpp"

namespace bpk {

hipError_t launch_sparse_sumf(const UpdateArgs& a, hipStream_t stream) {
    return dispatch_sparse<kSumF32>(a, stream);
}

hipError_t launch_sparse2_sumf(const UpdateArgs& a, hipStream_t stream) {
    return dispatch_sparse2<kSumF32>(a, stream);
}

}  // namespace bpk
