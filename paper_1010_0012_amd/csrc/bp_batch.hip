// Host driver of the batched path: instance descriptors, launch planning,
// concurrent launch chains, HIP graph capture and the plan autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/bp.h"
#include "bp_batch.hpp"
#include "bp_internal.hpp"
#include "bp_launch.hpp"

using namespace bpi;

struct bp_batch {
    int dev = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    int n = 0;
    std::vector<bp_grid_desc> desc;
    std::vector<int> arm;
    std::vector<float> fbar;
    // plan
    int passes[bpk::kBatchClasses] = {1, 1, 1, 1, 1};
    int grid_blocks = 0;
    // device memory: every instance's two message buffers
    char* ws = nullptr;
    int64_t ws_bytes = 0;
    size_t total = 0;
    std::vector<size_t> msg_bytes_off;        // per instance, first of its two buffers
    std::vector<bpk::InstDesc> hdesc;
    // launches: one or more per non-empty code path
    std::vector<bpk::BatchLaunch> launches;
    std::vector<int> launch_arm;
    std::vector<char> launch_full;       // every instance of the launch has M = 4G
    std::vector<char> launch_f32;        // sum-product of the launch in float32 arithmetic
    bool arith_f32 = false;              // BP_ARITH_F32 requested
    bool use_pairs = true;               // two iterations per launch (same bits as single launches)
    // Launches touch disjoint instances, so each launch's iterations form an
    // independent chain: the chains run on kSide streams (forked from and
    // joined back into the caller's stream by events), longest work first.
    static constexpr int kSide = 4;
    std::vector<int> launch_stream;
    int n_side = 0;                      // side streams in use (0: the caller's stream only)
    int max_streams = kSide;             // plan: launch chains on at most this many streams
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[kSide] = {};
    int parity = 0;
    bool use_graphs = true;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;  // (mode, n, parity)

    size_t msg_floats(int j) const { return (size_t)4 * desc[j].H * desc[j].W * desc[j].M; }
};

namespace {

// Lane class 0..4 for G = 4, 8, 16, 32, 64.
int lane_class(int M) {
    const int g = bpk::lanes_for(M);
    return g == 4 ? 0 : g == 8 ? 1 : g == 16 ? 2 : g == 32 ? 3 : 4;
}

// Smallest compiled code path whose window reaches T.
int pick_arm(int M, int T) {
    const int g = bpk::lanes_for(M);
    for (int a = 0; a < bpk::kBatchArms; ++a)
        if (bpk::arm_g(a) == g && bpk::arm_tw(a) >= T) return a;
    return -1;
}

void drop_graphs(bp_batch* B) {
    for (auto& kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
    B->graphs.clear();
}

bool full_rows(int M) { return M == bpk::lanes_for(M) * bpk::kLpl; }

// The row-block layout of a full launch (BatchLaunch.rows): per instance
// ceil(W / (kBlock/G)) workgroups per grid row, padded to a multiple of the
// XCD count; only when every inbox plane is below 2^32 bytes and the
// workgroup total fits an int.
void set_rows_layout(bpk::BatchLaunch& L) {
    L.rows = 0;
    long long end = 0;
    for (int k = 0; k < L.n_inst; ++k) {
        const bpk::InstDesc& d = L.inst[k];
        const int ppb = bpk::kBlock / bpk::lanes_for(d.M);
        if ((uint64_t)d.N * d.M * sizeof(float) >= (uint64_t(1) << 32)) return;
        L.gx[k] = (d.W + ppb - 1) / ppb;
        L.gxp[k] = (L.gx[k] + bpk::kXcds - 1) / bpk::kXcds * bpk::kXcds;
        end += (long long)L.gxp[k] * d.H;
        if (end >= (1LL << 31)) return;
        L.rows_end[k] = (int)end;
    }
    L.rows = 1;
}

// Launch plan: the instances of each code path (and whether M = 4G), largest
// first (bytes moved, pixels * M), packed into launches of up to
// kLaunchInst; each instance is cut into workgroups of passes * kBlock/G
// pixels (passes per lane class).  The launches are then spread over the
// side streams, longest first.
void build_launches(bp_batch* B) {
    B->launches.clear();
    B->launch_arm.clear();
    B->launch_full.clear();
    B->launch_f32.clear();
    std::vector<long long> work_of;
    auto work = [&](int j) { return (long long)B->desc[j].H * B->desc[j].W * B->desc[j].M; };
    for (int af = 0; af < 2 * bpk::kBatchArms; ++af) {
        const int a = af / 2;
        const bool full = af % 2 == 0;
        std::vector<int> js;
        for (int j = 0; j < B->n; ++j)
            if (B->arm[j] == a && full_rows(B->desc[j].M) == full) js.push_back(j);
        std::stable_sort(js.begin(), js.end(), [&](int x, int y) { return work(x) > work(y); });
        for (size_t i0 = 0; i0 < js.size(); i0 += bpk::kLaunchInst) {
            bpk::BatchLaunch L;
            memset(&L, 0, sizeof L);
            const int P = B->passes[lane_class(B->desc[js[i0]].M)];
            L.passes = P;
            long long w = 0;
            int blocks = 0;
            for (size_t i = i0; i < js.size() && i < i0 + bpk::kLaunchInst; ++i) {
                const int j = js[i];
                const int per_block = (bpk::kBlock / bpk::lanes_for(B->desc[j].M)) * P;
                blocks += (B->desc[j].H * B->desc[j].W + per_block - 1) / per_block;
                L.blocks_end[L.n_inst] = blocks;
                L.inst[L.n_inst] = B->hdesc[j];
                L.n_inst++;
                w += work(j);
            }
            if (full) set_rows_layout(L);
            // float32 arithmetic where the single-grid update has it: full
            // rows (the row-block layout) and fbar > 0 in every instance
            bool f32 = B->arith_f32 && full && L.rows;
            for (int k = 0; k < L.n_inst; ++k) f32 = f32 && L.inst[k].fbar > 0.0f;
            B->launches.push_back(L);
            B->launch_arm.push_back(a);
            B->launch_full.push_back(full);
            B->launch_f32.push_back(f32);
            work_of.push_back(w);
        }
    }
    const int nl = (int)B->launches.size();
    std::vector<int> order(nl);
    for (int i = 0; i < nl; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work_of[x] > work_of[y]; });
    const int ns = std::min(B->max_streams, nl);
    B->n_side = ns > 1 ? ns : 0;
    B->launch_stream.assign(nl, 0);
    long long load[bp_batch::kSide] = {};
    for (int l : order) {
        int best = 0;
        for (int i = 1; i < std::max(1, B->n_side); ++i)
            if (load[i] < load[best]) best = i;
        B->launch_stream[l] = best;
        load[best] += work_of[l];
    }
}

// Side streams and events, created on first use (default priority, like
// every stream this library touches).
hipError_t ensure_side(bp_batch* B) {
    if (B->ev_fork) return hipSuccess;
    hipError_t e = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming);
    for (int i = 0; i < bp_batch::kSide && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&B->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_join[i], hipEventDisableTiming);
    }
    return e;
}

unsigned launch_grid(const bp_batch* B, const bpk::BatchLaunch& L) {
    return (unsigned)std::max(1, std::min(B->grid_blocks, L.blocks_end[L.n_inst - 1]));
}

template <int MODE, int A = 0>
hipError_t launch_arm(int arm, const bpk::BatchLaunch& L, unsigned grid, int par, hipStream_t s) {
    if constexpr (A < bpk::kBatchArms) {
        if (arm != A) return launch_arm<MODE, A + 1>(arm, L, grid, par, s);
        if (L.passes == 1 && (int)grid == L.blocks_end[L.n_inst - 1])
            hipLaunchKernelGGL((bpk::batch_update_kernel<MODE, bpk::arm_g(A), bpk::arm_tw(A), false>), dim3(grid),
                               dim3(bpk::kBlock), 0, s, L, par);
        else
            hipLaunchKernelGGL((bpk::batch_update_kernel<MODE, bpk::arm_g(A), bpk::arm_tw(A), true>), dim3(grid),
                               dim3(bpk::kBlock), 0, s, L, par);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

// Launches per entry of the plan for n iterations: with pairs, n / 2
// two-iteration launches and a single one for an odd n.  Each launch flips
// the buffer parity once.
int launches_for(const bp_batch* B, int n) { return B->use_pairs ? n / 2 + (n & 1) : n; }

// n iterations: per iteration (or pair of iterations) one launch per entry
// of the plan.  The launches touch disjoint instances, so their chains run
// concurrently on the side streams, forked from s after the work already
// queued there and joined back into s.
hipError_t launch_iters(bp_batch* B, int mode, int n, int parity0, hipStream_t s) {
    hipError_t e = hipSuccess;
    const bool fork = B->n_side > 1;
    if (fork) {
        if ((e = ensure_side(B)) != hipSuccess) return e;
        if ((e = hipEventRecord(B->ev_fork, s)) != hipSuccess) return e;
        for (int i = 0; i < B->n_side; ++i)
            if ((e = hipStreamWaitEvent(B->side[i], B->ev_fork, 0)) != hipSuccess) return e;
    }
    const int pairs = B->use_pairs ? n / 2 : 0;
    for (int t = 0; t < launches_for(B, n); ++t) {
        const int par = (parity0 + t) & 1;
        for (size_t l = 0; l < B->launches.size(); ++l) {
            const bpk::BatchLaunch& L = B->launches[l];
            hipStream_t ls = fork ? B->side[B->launch_stream[l]] : s;
            const int arm = B->launch_arm[l];
            const unsigned grid = launch_grid(B, L);
            const bool f32 = mode == bpk::kSum && B->launch_f32[l];
            if (t < pairs)
                e = f32                   ? bpk::launch_batch_pair_sumf(arm, B->launch_full[l], L, grid, par, ls)
                    : mode == bpk::kSum ? bpk::launch_batch_pair_sum(arm, B->launch_full[l], L, grid, par, ls)
                                        : bpk::launch_batch_pair_max(arm, B->launch_full[l], L, grid, par, ls);
            else
                e = f32                   ? launch_arm<bpk::kSumF32>(arm, L, grid, par, ls)
                    : mode == bpk::kSum ? launch_arm<bpk::kSum>(arm, L, grid, par, ls)
                                        : launch_arm<bpk::kMax>(arm, L, grid, par, ls);
            if (e != hipSuccess) return e;
        }
    }
    if (fork) {
        for (int i = 0; i < B->n_side; ++i) {
            if ((e = hipEventRecord(B->ev_join[i], B->side[i])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, B->ev_join[i], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int ready(const bp_batch* B) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    if (!B->ws) return fail(BP_ESTATE, "no workspace attached to the batch");
    return BP_OK;
}

int set_device(const bp_batch* B) {
    hipError_t e = hipSetDevice(B->dev);
    return e == hipSuccess ? BP_OK : hip_fail(e, "hipSetDevice");
}

}  // namespace

extern "C" {

int bp_batch_init(bp_batch** out, int32_t n, const bp_grid_desc* descs, void* hip_stream) {
    if (!out) return fail(BP_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (n < 1 || !descs) return fail(BP_EINVAL, "need n >= 1 descriptors");
    std::vector<int> arms(n);
    std::vector<float> fbars(n);
    for (int j = 0; j < n; ++j) {
        const bp_grid_desc& d = descs[j];
        if (d.H < 1 || d.W < 1 || (int64_t)d.H * d.W >= (int64_t(1) << 29))
            return fail(BP_EINVAL, "instance %d: bad grid %d x %d", j, d.H, d.W);
        if (d.M < 1 || d.T < 0 || d.T >= d.M) return fail(BP_EINVAL, "instance %d: need 1 <= M and 0 <= T < M", j);
        if (d.M > BP_MAX_LABELS || d.T > 8)
            return fail(BP_EUNSUPPORTED, "instance %d: batches support M <= %d, T <= 8", j, BP_MAX_LABELS);
        if (!std::isfinite(d.alpha)) return fail(BP_EINVAL, "instance %d: alpha not finite", j);
        float fb = d.fbar;
        if (fb == BP_FBAR_TIED) fb = (float)std::exp(-(double)d.alpha * d.T);
        if (!std::isfinite(fb) || fb < 0.0f) return fail(BP_EINVAL, "instance %d: bad fbar", j);
        if (!d.unary || reinterpret_cast<uintptr_t>(d.unary) % 16)
            return fail(BP_EINVAL, "instance %d: unary null or not 16-byte aligned", j);
        arms[j] = pick_arm(d.M, d.T);
        if (arms[j] < 0) return fail(BP_EUNSUPPORTED, "instance %d: no compiled window for M=%d T=%d", j, d.M, d.T);
        fbars[j] = fb;
    }
    int dev = -1;  // after the host-side checks: argument errors are reported as such without a device
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    bp_batch* B = new (std::nothrow) bp_batch();
    if (!B) return fail(BP_ENOMEM, "host allocation failed");
    B->dev = dev;
    B->stream = static_cast<hipStream_t>(hip_stream);
    B->n = n;
    B->desc.assign(descs, descs + n);
    B->arm = arms;
    B->fbar = fbars;
    B->grid_blocks = 1 << 30;  // one workgroup per pixel range until a plan says otherwise
    size_t off = 0;
    for (int j = 0; j < n; ++j) {
        B->msg_bytes_off.push_back(off);
        off += 2 * bp_align_up(B->msg_floats(j) * sizeof(float), 256);
    }
    B->total = off;
    BP_ASSERT(B->msg_bytes_off.size() == (size_t)n && (n == 0 || B->msg_bytes_off.back() < off));
    *out = B;
    return BP_OK;
}

int bp_batch_set_stream(bp_batch* B, void* hip_stream) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    B->stream = static_cast<hipStream_t>(hip_stream);
    return BP_OK;
}

int64_t bp_batch_workspace_bytes(const bp_batch* B) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    return (int64_t)B->total;
}

int bp_batch_attach_workspace(bp_batch* B, void* dev_ptr, int64_t bytes) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    if (!dev_ptr) return fail(BP_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(BP_EINVAL, "workspace not 256-byte aligned");
    if (bytes < (int64_t)B->total)
        return fail(BP_ENOMEM, "workspace %lld bytes < %zu needed", (long long)bytes, B->total);
    // the instance descriptors (host), then the device
    char* ws = static_cast<char*>(dev_ptr);
    std::vector<bpk::InstDesc> hdesc(B->n, bpk::InstDesc{});
    long long boff = 0, loff = 0;
    for (int j = 0; j < B->n; ++j) {
        const bp_grid_desc& d = B->desc[j];
        bpk::InstDesc& h = hdesc[j];
        memset(&h, 0, sizeof h);
        h.g = d.unary;
        const size_t buf = bp_align_up(B->msg_floats(j) * sizeof(float), 256);
        BP_ASSERT(B->msg_bytes_off[j] + 2 * buf <= (size_t)bytes);
        BP_ASSERT(j + 1 == B->n || B->msg_bytes_off[j] + 2 * buf == B->msg_bytes_off[j + 1]);
        h.msg[0] = reinterpret_cast<float*>(ws + B->msg_bytes_off[j]);
        h.msg[1] = reinterpret_cast<float*>(ws + B->msg_bytes_off[j] + buf);
        h.belief_off = boff;
        h.label_off = loff;
        h.H = d.H; h.W = d.W; h.M = d.M; h.N = d.H * d.W; h.T = d.T;
        h.arm = B->arm[j];
        h.fbar = B->fbar[j];
        h.fbar_d = d.fbar == BP_FBAR_TIED ? std::exp(-(double)d.alpha * d.T) : (double)d.fbar;
        for (int k = 0; k < bpk::kBatchTab; ++k) {
            const bool in = k <= d.T;
            const double f = std::exp(-(double)d.alpha * k);
            h.tab_f[k] = in ? (float)f : 0.0f;
            h.tab_wf[k] = in ? (float)(f - (double)h.fbar) : 0.0f;
            h.tab_wd[k] = in ? f - h.fbar_d : 0.0;
        }
        boff += (long long)h.N * d.M;
        loff += h.N;
    }
    int st = set_device(B);
    if (st) return st;
    drop_graphs(B);
    B->ws = ws;
    B->ws_bytes = bytes;
    B->hdesc.swap(hdesc);
    build_launches(B);
    return bp_batch_reset_messages(B);
}

int bp_batch_reset_messages(bp_batch* B) {
    int st = ready(B);
    if (st) return st;
    if ((st = set_device(B))) return st;
    for (int j = 0; j < B->n; ++j)
        for (int b = 0; b < 2; ++b) {
            hipError_t e = bpk::launch_fill(B->hdesc[j].msg[b], B->msg_floats(j), 1.0f / (float)B->desc[j].M, B->stream);
            if (e != hipSuccess) return hip_fail(e, "batch message reset");
        }
    B->parity = 0;
    return BP_OK;
}

int bp_batch_iterate(bp_batch* B, int32_t mode, int32_t n_iters) {
    TraceRange tr("bp_batch_iterate");
    int st = ready(B);
    if (st) return st;
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (n_iters < 0) return fail(BP_EINVAL, "n_iters < 0");
    if (mode == BP_MAX_PRODUCT)
        for (int j = 0; j < B->n; ++j)
            for (int d = 0; d <= B->desc[j].T; ++d)
                if (!(B->hdesc[j].tab_f[d] >= B->hdesc[j].fbar))
                    return fail(BP_EUNSUPPORTED, "instance %d: max-product needs f >= fbar (Eq. 11)", j);
    if (n_iters == 0) return BP_OK;
    if ((st = set_device(B))) return st;
    const int kmode = mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax;
    hipError_t e;
    if (!B->use_graphs) {
        e = launch_iters(B, kmode, n_iters, B->parity, B->stream);
        if (e != hipSuccess) return hip_fail(e, "batch update launch");
    } else {
        const auto key = std::make_tuple(kmode, (int)n_iters, B->parity);
        auto it = B->graphs.find(key);
        if (it == B->graphs.end()) {
            if (!B->cap_stream) {
                // default priority, like every stream this library touches
                e = hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "capture stream");
            }
            e = hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = launch_iters(B, kmode, n_iters, B->parity, B->cap_stream);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(B->cap_stream, &graph);
            if (le != hipSuccess) return hip_fail(le, "batch update capture");
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            it = B->graphs.emplace(key, exec).first;
        }
        e = hipGraphLaunch(it->second, B->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    B->parity ^= launches_for(B, n_iters) & 1;
    return BP_OK;
}

int bp_batch_set_arithmetic(bp_batch* B, int32_t arith) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    if (arith != BP_ARITH_F64 && arith != BP_ARITH_F32) return fail(BP_EINVAL, "bad arithmetic %d", arith);
    if ((arith == BP_ARITH_F32) == B->arith_f32) return BP_OK;
    drop_graphs(B);
    B->arith_f32 = arith == BP_ARITH_F32;
    if (B->ws) build_launches(B);
    return BP_OK;
}

int bp_batch_set_graphs(bp_batch* B, int32_t enable) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    B->use_graphs = enable != 0;
    return BP_OK;
}

int bp_batch_set_plan(bp_batch* B, const int32_t passes[5], int32_t grid_blocks) {
    int st = ready(B);
    if (st) return st;
    if (!passes || grid_blocks < 1) return fail(BP_EINVAL, "bad plan");
    for (int c = 0; c < bpk::kBatchClasses; ++c)
        if (passes[c] < 1 || passes[c] > 4096) return fail(BP_EINVAL, "passes[%d] out of range", c);
    drop_graphs(B);
    for (int c = 0; c < bpk::kBatchClasses; ++c) B->passes[c] = passes[c];
    B->grid_blocks = grid_blocks;
    build_launches(B);
    return BP_OK;
}

int bp_batch_set_streams(bp_batch* B, int32_t n_streams) {
    int st = ready(B);
    if (st) return st;
    if (n_streams < 1 || n_streams > bp_batch::kSide) return fail(BP_EINVAL, "n_streams must be in [1, %d]", bp_batch::kSide);
    drop_graphs(B);
    B->max_streams = n_streams;
    build_launches(B);
    return BP_OK;
}

int bp_batch_get_streams(const bp_batch* B) {
    if (!B) return fail(BP_EINVAL, "null batch handle");
    return B->max_streams;
}

int bp_batch_get_plan(const bp_batch* B, int32_t passes[5], int32_t* grid_blocks) {
    if (!B || !passes || !grid_blocks) return fail(BP_EINVAL, "null argument");
    for (int c = 0; c < bpk::kBatchClasses; ++c) passes[c] = B->passes[c];
    *grid_blocks = B->grid_blocks;
    return BP_OK;
}

int bp_batch_autotune(bp_batch* B, int32_t mode, int32_t trial_iters, float* best_us) {
    int st = ready(B);
    if (st) return st;
    if (mode != BP_SUM_PRODUCT && mode != BP_MAX_PRODUCT) return fail(BP_EINVAL, "bad mode %d", mode);
    if (trial_iters < 1) return fail(BP_EINVAL, "trial_iters must be >= 1");
    if ((st = set_device(B))) return st;
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    const int kmode = mode == BP_SUM_PRODUCT ? bpk::kSum : bpk::kMax;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
    // Candidates: launch chains on one stream or on all side streams, times
    // workgroups of 1/2/4/8 passes (a pass moves about the same bytes in
    // every lane class), times persistent grid sizes of 2..16 workgroups per
    // CU, and one workgroup per pixel range.
    struct Cand { int streams, scale, grid; };
    std::vector<Cand> cands;
    for (int streams : {1, bp_batch::kSide})
        for (int scale : {1, 2, 4, 8})
            for (int per_cu : {2, 4, 8, 16, 0})
                cands.push_back({streams, scale, per_cu ? std::max(1, cus) * per_cu : (1 << 30)});
    float best = 1e30f;
    Cand best_c = {bp_batch::kSide, 1, 1 << 30};
    for (const Cand& c : cands) {
        int32_t pl[bpk::kBatchClasses];
        for (int k = 0; k < bpk::kBatchClasses; ++k) pl[k] = c.scale;
        B->max_streams = c.streams;
        if ((st = bp_batch_set_plan(B, pl, c.grid))) break;
        e = launch_iters(B, kmode, 1, B->parity, B->stream);  // warm
        if (e == hipSuccess) e = hipEventRecord(e0, B->stream);
        if (e == hipSuccess) e = launch_iters(B, kmode, trial_iters, B->parity ^ 1, B->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, B->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = hip_fail(e, "autotune trial"); break; }
        B->parity ^= (launches_for(B, 1) + launches_for(B, trial_iters)) & 1;
        const float us = ms * 1000.0f / trial_iters;
        if (us < best) {
            best = us;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    B->max_streams = best_c.streams;
    int32_t best_passes[bpk::kBatchClasses];
    for (int k = 0; k < bpk::kBatchClasses; ++k) best_passes[k] = best_c.scale;
    if ((st = bp_batch_set_plan(B, best_passes, best_c.grid))) return st;
    if (best_us) *best_us = best;
    return bp_batch_reset_messages(B);
}

static int batch_readout(bp_batch* B, float* beliefs, int32_t* labels) {
    int st = ready(B);
    if (st) return st;
    if ((st = set_device(B))) return st;
    for (size_t l = 0; l < B->launches.size(); ++l) {
        const bpk::BatchLaunch& L = B->launches[l];
        const unsigned grid = launch_grid(B, L);
        switch (bpk::arm_g(B->launch_arm[l])) {
            case 4: hipLaunchKernelGGL(bpk::batch_readout_kernel<4>, dim3(grid), dim3(bpk::kBlock), 0, B->stream,
                                       L, B->parity, beliefs, labels); break;
            case 8: hipLaunchKernelGGL(bpk::batch_readout_kernel<8>, dim3(grid), dim3(bpk::kBlock), 0, B->stream,
                                       L, B->parity, beliefs, labels); break;
            case 16: hipLaunchKernelGGL(bpk::batch_readout_kernel<16>, dim3(grid), dim3(bpk::kBlock), 0, B->stream,
                                        L, B->parity, beliefs, labels); break;
            case 32: hipLaunchKernelGGL(bpk::batch_readout_kernel<32>, dim3(grid), dim3(bpk::kBlock), 0, B->stream,
                                        L, B->parity, beliefs, labels); break;
            default: hipLaunchKernelGGL(bpk::batch_readout_kernel<64>, dim3(grid), dim3(bpk::kBlock), 0, B->stream,
                                        L, B->parity, beliefs, labels); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "batch readout launch");
    }
    return BP_OK;
}

int bp_batch_beliefs(bp_batch* B, float* out_dev) {
    if (!out_dev || reinterpret_cast<uintptr_t>(out_dev) % 16) return fail(BP_EINVAL, "beliefs output null or misaligned");
    return batch_readout(B, out_dev, nullptr);
}

int bp_batch_map_labels(bp_batch* B, int32_t* out_dev) {
    if (!out_dev) return fail(BP_EINVAL, "null labels output");
    return batch_readout(B, nullptr, out_dev);
}

int bp_batch_destroy(bp_batch* B) {
    if (!B) return BP_OK;
    drop_graphs(B);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    for (int i = 0; i < bp_batch::kSide; ++i) {
        if (B->side[i]) (void)hipStreamDestroy(B->side[i]);
        if (B->ev_join[i]) (void)hipEventDestroy(B->ev_join[i]);
    }
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    delete B;
    return BP_OK;
}

}  // extern "C"
