// bp_solve_noalloc: a whole single-grid solve for callers that cannot
// allocate device memory (code under stream capture, serving loops, harnesses
// that forbid allocation).  The message buffers live in a file-scope device
// array of fixed size instead of a caller-attached workspace; the handle state
// lives on the host stack.  Nothing here allocates device or host memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bp.h"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using namespace bpi;

namespace {

constexpr size_t kStaticBytes = BP_NOALLOC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

// Every GPU the library runs on holds one copy until the process ends.
static __device__ __align__(256) char scratch[kStaticBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this GPU's scratch array (looked up once per device,
// with that device current): host code must never pass the array's own name,
// which is a host-side stand-in, to a kernel or a copy.
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(BP_EUNSUPPORTED, "device %d beyond the static table", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static workspace)");
        if (!p) return fail(BP_EHIP, "hipGetSymbolAddress returned null");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return BP_OK;
}

}  // namespace

extern "C" {

int bp_solve_noalloc(const float* g_dev, int32_t H, int32_t W, int32_t M, int32_t T, float alpha, float fbar,
                     int32_t mode, int32_t n_iters, int32_t schedule, float* beliefs_dev, int32_t* labels_dev,
                     void* hip_stream) {
    if (H < 1 || W < 1) return fail(BP_EINVAL, "grid %d x %d: both sides must be >= 1", H, W);
    if ((int64_t)H * W >= (int64_t(1) << 29)) return fail(BP_EINVAL, "grid too large");
    if (!beliefs_dev && !labels_dev) return fail(BP_EINVAL, "null beliefs and labels outputs");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    bp_grid G;  // host stack: no handle allocation
    G.dev = dev;
    G.stream = static_cast<hipStream_t>(hip_stream);
    G.H = H;
    G.W = W;
    G.N = H * W;
    int st = bp_set_potential(&G, M, T, alpha, fbar);
    if (st) return st;
    const int64_t need = bp_workspace_bytes(&G);
    if (need < 0) return (int)need;
    if ((uint64_t)need > kStaticBytes)
        return fail(BP_EINVAL, "H*W*M = %lld needs %lld bytes of messages and tables; the static workspace holds %zu",
                    (long long)G.N * M, (long long)need, kStaticBytes);
    // Max-product with fbar above f(T) beyond the register windows runs the
    // general kernel on tables staged through host memory: not here.
    if (mode == BP_MAX_PRODUCT && !max_product_ok(&G) && bpk::sparse_variant_tw(M, T) < 0)
        return fail(BP_EUNSUPPORTED, "Eq. 10 max-product with T=%d beyond the register windows (M=%d)", T, M);
    void* ws = nullptr;
    if ((st = scratch_ptr(dev, &ws))) return st;
    // attach resets every message to 1/M (fill kernels, the whole state)
    if ((st = bp_attach_workspace(&G, ws, (int64_t)kStaticBytes))) return st;
    if ((st = bp_set_unary(&G, g_dev))) return st;
    if ((st = bp_iterate(&G, mode, n_iters, schedule))) return st;
    return bp_readout(&G, beliefs_dev, labels_dev);
}

}  // extern "C"
