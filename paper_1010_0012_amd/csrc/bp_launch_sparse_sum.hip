// Sparse O(mM) sum-product update (Eq. 7): instantiations and dispatch.
#include "bp_sparse_dispatch.hpp"

namespace bpk {

hipError_t launch_sparse_max(const UpdateArgs& a, hipStream_t stream);  // bp_launch_sparse_max.hip

int sparse_variant_tw(int M, int T) { return sparse_tw(M, T); }

hipError_t launch_sparse(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    return mode == kSum ? dispatch_sparse<kSum>(a, stream) : launch_sparse_max(a, stream);
}

}  // namespace bpk
