// Sparse O(mM) sum-product update (Eq. 7): instantiations and dispatch.
#include "bp_sparse_dispatch.hpp"

namespace bpk {

hipError_t launch_sparse_max(const UpdateArgs& a, hipStream_t stream);   // bp_launch_sparse_max.hip
hipError_t launch_sparse2_max(const UpdateArgs& a, hipStream_t stream);  // bp_launch_sparse_max.hip
hipError_t launch_sparse_sumf(const UpdateArgs& a, hipStream_t stream);   // bp_launch_sparse_sumf.hip
hipError_t launch_sparse2_sumf(const UpdateArgs& a, hipStream_t stream);  // bp_launch_sparse_sumf.hip

int sparse_variant_tw(int M, int T) { return sparse_tw(M, T); }

hipError_t launch_sparse(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    if (mode == kSumF32) return launch_sparse_sumf(a, stream);
    return mode == kSum ? dispatch_sparse<kSum>(a, stream) : launch_sparse_max(a, stream);
}

bool sparse2_supported(int M, int T) { return sparse_tw(M, T) >= 0; }

hipError_t launch_sparse2(const UpdateArgs& a, int mode, hipStream_t stream) {
    if (a.n_slots <= 0) return hipSuccess;
    if (mode == kSumF32) return launch_sparse2_sumf(a, stream);
    return mode == kSum ? dispatch_sparse2<kSum>(a, stream) : launch_sparse2_max(a, stream);
}

}  // namespace bpk
