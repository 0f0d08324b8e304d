// Sparse O(mM) max-product update (Eq. 11): instantiations and dispatch.
#include "bp_sparse_dispatch.hpp"

namespace bpk {

hipError_t launch_sparse_max(const UpdateArgs& a, hipStream_t stream) {
    return dispatch_sparse<kMax>(a, stream);
}

hipError_t launch_sparse2_max(const UpdateArgs& a, hipStream_t stream) {
    return dispatch_sparse2<kMax>(a, stream);
}

}  // namespace bpk
