// Host-side runtime of libbp_hip under AddressSanitizer and
// UndefinedBehaviorSanitizer, with the library's BP_DEBUG checks compiled in:
// every entry point's argument checks, the potential tables, the workspace,
// gradient, multi-scale and sparse-table layouts, batch descriptor checks
// and the factor-graph build, all of which run before the first device
// call.  Built and run on a machine without a GPU (every device call then
// fails cleanly with BP_EHIP); it refuses to run where a GPU is present,
// since it hands the library host addresses in place of device buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bp.h"
#include "bp_internal.hpp"

static int failures = 0;
static int checks = 0;

#define EXPECT(cond)                                                                                   \
    do {                                                                                               \
        ++checks;                                                                                      \
        if (!(cond)) {                                                                                 \
            std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", __LINE__, #cond, bp_last_error()); \
            ++failures;                                                                                \
        }                                                                                              \
    } while (0)

// A 256-byte-aligned host block standing in for a device buffer of any
// size: the host code only checks and offsets such pointers, and the device
// calls that would use them fail first on a machine without a GPU.
alignas(4096) static char g_fake[4096];
static void* fake_device(size_t) { return g_fake; }

static void null_handles() {
    float f = 0.0f;
    int32_t i = 0;
    EXPECT(bp_set_stream(nullptr, nullptr) == BP_EINVAL);
    EXPECT(bp_set_potential(nullptr, 8, 2, 1.0f, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_workspace_bytes(nullptr) == BP_EINVAL);
    EXPECT(bp_attach_workspace(nullptr, &f, 4) == BP_EINVAL);
    EXPECT(bp_set_unary(nullptr, &f) == BP_EINVAL);
    EXPECT(bp_reset_messages(nullptr) == BP_EINVAL);
    EXPECT(bp_iterate(nullptr, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC) == BP_EINVAL);
    EXPECT(bp_iterate_dense(nullptr, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC) == BP_EINVAL);
    EXPECT(bp_set_sync_fusion(nullptr, 1) == BP_EINVAL);
    EXPECT(bp_set_arithmetic(nullptr, BP_ARITH_F32) == BP_EINVAL);
    EXPECT(bp_set_launch_tuning(nullptr, BP_PAIR_STRIPS, -1) == BP_EINVAL);
    EXPECT(bp_get_launch_tuning(nullptr, &i, &i) == BP_EINVAL);
    EXPECT(bp_autotune(nullptr, BP_SUM_PRODUCT, BP_SCHED_SYNC, 2, &f) == BP_EINVAL);
    EXPECT(bp_batch_set_arithmetic(nullptr, BP_ARITH_F32) == BP_EINVAL);
    EXPECT(bp_beliefs(nullptr, &f) == BP_EINVAL);
    EXPECT(bp_map_labels(nullptr, &i) == BP_EINVAL);
    EXPECT(bp_readout(nullptr, nullptr, nullptr) == BP_EINVAL);
    EXPECT(bp_get_messages(nullptr, &f) == BP_EINVAL);
    EXPECT(bp_set_messages(nullptr, &f) == BP_EINVAL);
    EXPECT(bp_grad_workspace_bytes(nullptr, 3, 1) == BP_EINVAL);
    EXPECT(bp_forward_ckpt(nullptr, 3, 1, &f, 4) == BP_EINVAL);
    EXPECT(bp_backward(nullptr, &f, &f, &f) == BP_EINVAL);
    EXPECT(bp_sparse_table_bytes(nullptr, 1, nullptr) == BP_EINVAL);
    EXPECT(bp_multiscale_workspace_bytes(nullptr, 1) == BP_EINVAL);
    EXPECT(bp_iterate_multiscale(nullptr, BP_SUM_PRODUCT, 0, &i, nullptr, 0) == BP_EINVAL);
    EXPECT(bp_destroy(nullptr) == BP_EINVAL || bp_destroy(nullptr) == BP_OK);
    EXPECT(bp_batch_set_stream(nullptr, nullptr) == BP_EINVAL);
    EXPECT(bp_batch_workspace_bytes(nullptr) == BP_EINVAL);
    EXPECT(bp_batch_attach_workspace(nullptr, &f, 4) == BP_EINVAL);
    EXPECT(bp_batch_iterate(nullptr, BP_SUM_PRODUCT, 1) < 0);
    EXPECT(bp_batch_get_streams(nullptr) < 0);
    EXPECT(bp_fg_workspace_bytes(nullptr) < 0);
    EXPECT(bp_fg_attach_workspace(nullptr, &f, 4) < 0);
    EXPECT(bp_fg_iterate(nullptr, BP_SUM_PRODUCT, 1, 0) < 0);
    for (int s = 0; s >= -6; --s) EXPECT(bp_status_string(s) != nullptr);
}

static void init_without_device() {
    bp_grid* h = reinterpret_cast<bp_grid*>(1);
    EXPECT(bp_init_grid(nullptr, 4, 4, nullptr) == BP_EINVAL);
    EXPECT(bp_init_grid(&h, 0, 4, nullptr) == BP_EINVAL && h == nullptr);
    EXPECT(bp_init_grid(&h, 4, -1, nullptr) == BP_EINVAL);
    EXPECT(bp_init_grid(&h, 1 << 15, 1 << 15, nullptr) == BP_EINVAL);
    EXPECT(bp_init_grid(&h, 4, 4, nullptr) == BP_EHIP && h == nullptr);
}

// A grid handle built on the host (no device), as bp_init_grid would leave it.
static void host_grid(bp_grid& G, int H, int W) {
    G.dev = 0;
    G.H = H;
    G.W = W;
    G.N = H * W;
}

static void potentials_and_layouts() {
    const int sizes[][2] = {{1, 1}, {1, 9}, {7, 1}, {5, 6}, {33, 17}, {480, 640}};
    const int labels[] = {1, 2, 5, 16, 20, 33, 64, 100, 128, 200, 256};
    for (auto& hw : sizes)
        for (int M : labels)
            for (int T : {0, 1, M / 2, M - 1}) {
                if (T < 0 || T >= M) continue;
                bp_grid G;
                host_grid(G, hw[0], hw[1]);
                EXPECT(bp_set_potential(&G, M, T, 0.7f, BP_FBAR_TIED) == BP_OK);
                for (int d = 0; d <= T && d < bpk::kMaxTab; ++d) EXPECT(G.tab_f[d] >= G.fbar);
                const int64_t ws = bp_workspace_bytes(&G);
                EXPECT(ws > 0 && ws % 256 == 0 && ws >= (int64_t)(8 * G.msg_floats()));
                for (int n : {0, 1, 5, 30})
                    for (int k : {1, 2, 5, 40}) {
                        const int64_t g = bp_grad_workspace_bytes(&G, n, k);
                        EXPECT(g > 0 && g % 256 == 0);
                    }
                for (int l = 0; l <= 4; ++l) EXPECT(bp_multiscale_workspace_bytes(&G, l) >= 256);
                EXPECT(bp_multiscale_workspace_bytes(&G, -1) == BP_EINVAL);
                // the workspace carving runs; the reset's device call then fails
                void* w = fake_device((size_t)ws);
                EXPECT(bp_attach_workspace(&G, w, ws - 1) == BP_ENOMEM);
                EXPECT(bp_attach_workspace(&G, static_cast<char*>(w) + 16, ws) == BP_EINVAL);
                EXPECT(bp_attach_workspace(&G, w, ws) == BP_EHIP);
                EXPECT(bp_set_arithmetic(&G, BP_ARITH_F32) == BP_OK && G.arith_f32);
                EXPECT(bp_set_arithmetic(&G, 7) == BP_EINVAL && G.arith_f32);
                EXPECT(bp_set_arithmetic(&G, BP_ARITH_F64) == BP_OK && !G.arith_f32);
                {
                    int32_t lay = -7, cap = -7;
                    EXPECT(bp_get_launch_tuning(&G, &lay, &cap) == BP_OK && lay == BP_PAIR_WIDE && cap == -1);
                    // the default mapping follows the arithmetic until one is chosen
                    EXPECT(bp_set_arithmetic(&G, BP_ARITH_F32) == BP_OK && G.pair_layout == BP_PAIR_TILE);
                    EXPECT(bp_set_arithmetic(&G, BP_ARITH_F64) == BP_OK && G.pair_layout == BP_PAIR_WIDE);
                    EXPECT(bp_set_launch_tuning(&G, BP_PAIR_SLOTS, 3) == BP_OK);
                    EXPECT(bp_get_launch_tuning(&G, &lay, &cap) == BP_OK && lay == BP_PAIR_SLOTS && cap == 3);
                    EXPECT(bp_set_launch_tuning(&G, 6, 0) == BP_EINVAL && G.pair_layout == BP_PAIR_SLOTS);
                    EXPECT(bp_set_launch_tuning(&G, BP_PAIR_BANDS, 65) == BP_EINVAL && G.pair_cap == 3);
                    EXPECT(bp_get_launch_tuning(&G, nullptr, &cap) == BP_EINVAL);
                    // not ready (no unary): refused before any device work
                    EXPECT(bp_autotune(&G, BP_SUM_PRODUCT, BP_SCHED_SYNC, 2, nullptr) == BP_ESTATE);
                    EXPECT(bp_set_arithmetic(&G, BP_ARITH_F32) == BP_OK && G.pair_layout == BP_PAIR_SLOTS);
                    EXPECT(bp_set_arithmetic(&G, BP_ARITH_F64) == BP_OK && G.pair_layout == BP_PAIR_SLOTS);
                    EXPECT(bp_set_launch_tuning(&G, BP_PAIR_WIDE, -1) == BP_OK);
                }
                // other potentials on the same handle
                EXPECT(bp_set_potential(&G, M, T, 1.5f, 0.0f) == BP_OK);
                EXPECT(bp_set_potential(&G, M, T, -0.3f, 0.5f) == BP_OK);
            }
    bp_grid G;
    host_grid(G, 4, 5);
    EXPECT(bp_set_potential(&G, 0, 0, 1.0f, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, BP_MAX_LABELS + 1, 2, 1.0f, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, 8, 8, 1.0f, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, 8, -1, 1.0f, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, 8, 2, NAN, BP_FBAR_TIED) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, 8, 2, 1.0f, -2.0f) == BP_EINVAL);
    EXPECT(bp_set_potential(&G, 8, 2, 1.0f, INFINITY) == BP_EINVAL);
    bp_grid U;
    host_grid(U, 4, 5);
    EXPECT(bp_workspace_bytes(&U) == BP_ESTATE);
    EXPECT(bp_iterate(&U, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC) == BP_ESTATE);
}

static void sparse_tables() {
    std::srand(7);
    for (int M : {3, 16, 64, 200}) {
        bp_grid G;
        host_grid(G, 6, 7);
        EXPECT(bp_set_potential(&G, M, 1, 1.0f, BP_FBAR_TIED) == BP_OK);
        std::vector<int32_t> ptr(M + 1, 0), idx;
        std::vector<float> val;
        for (int y = 0; y < M; ++y) {
            for (int x = 0; x < M; ++x)
                if (x == y || std::rand() % 5 == 0) {
                    idx.push_back(x);
                    val.push_back(0.1f + (float)(std::rand() % 100) / 100.0f);
                }
            ptr[y + 1] = (int32_t)idx.size();
        }
        bp_sparse_potential t{ptr.data(), idx.data(), val.data(), 0.05f};
        bp_sparse_potential four[4] = {t, t, t, t};
        const int64_t b1 = bp_sparse_table_bytes(&G, 1, &t);
        const int64_t b4 = bp_sparse_table_bytes(&G, 4, four);
        EXPECT(b1 > 0 && b4 >= b1 && b1 % 256 == 0);
        EXPECT(bp_sparse_table_bytes(&G, 0, &t) == BP_EINVAL);
        EXPECT(bp_set_sparse_potentials(&G, 1, &t, fake_device((size_t)b1), b1 - 1, nullptr, nullptr) == BP_ENOMEM);
        EXPECT(bp_set_sparse_potentials(&G, 1, &t, fake_device((size_t)b1), b1, nullptr, nullptr) == BP_EHIP);
        // broken tables
        std::vector<int32_t> bad = idx;
        for (int y = 0; y < M; ++y)
            if (ptr[y + 1] - ptr[y] >= 2) {  // two labels of one column out of order
                std::swap(bad[ptr[y]], bad[ptr[y] + 1]);
                bp_sparse_potential u{ptr.data(), bad.data(), val.data(), 0.05f};
                EXPECT(bp_sparse_table_bytes(&G, 1, &u) == BP_EINVAL);
                break;
            }
        bad = idx;
        bad.back() = M;
        bp_sparse_potential v{ptr.data(), bad.data(), val.data(), 0.05f};
        EXPECT(bp_sparse_table_bytes(&G, 1, &v) == BP_EINVAL);
        std::vector<float> neg = val;
        neg[0] = -1.0f;
        bp_sparse_potential w{ptr.data(), idx.data(), neg.data(), 0.05f};
        EXPECT(bp_sparse_table_bytes(&G, 1, &w) == BP_EINVAL);
        bp_sparse_potential z{ptr.data(), idx.data(), val.data(), NAN};
        EXPECT(bp_sparse_table_bytes(&G, 1, &z) == BP_EINVAL);
    }
}

static void batches() {
    void* g = fake_device(1 << 20);
    std::vector<bp_grid_desc> d;
    for (int j = 0; j < 12; ++j) {
        const int M = (int[]){16, 32, 64, 128}[j % 4];
        d.push_back(bp_grid_desc{3 + 7 * j, 5 + 3 * j, M, 1 + j % 8, 0.3f + 0.1f * j, BP_FBAR_TIED,
                                 static_cast<float*>(g)});
    }
    bp_batch* B = nullptr;
    EXPECT(bp_batch_init(&B, (int32_t)d.size(), d.data(), nullptr) == BP_EHIP && B == nullptr);
    EXPECT(bp_batch_init(nullptr, 1, d.data(), nullptr) == BP_EINVAL);
    EXPECT(bp_batch_init(&B, 0, d.data(), nullptr) == BP_EINVAL);
    std::vector<bp_grid_desc> e = d;
    e[3].T = e[3].M;
    EXPECT(bp_batch_init(&B, (int32_t)e.size(), e.data(), nullptr) == BP_EINVAL);
    e = d;
    e[5].unary = static_cast<float*>(g) + 1;
    EXPECT(bp_batch_init(&B, (int32_t)e.size(), e.data(), nullptr) == BP_EINVAL);
    e = d;
    e[2].T = 9;
    EXPECT(bp_batch_init(&B, (int32_t)e.size(), e.data(), nullptr) == BP_EUNSUPPORTED);
    e = d;
    e[0].alpha = NAN;
    EXPECT(bp_batch_init(&B, (int32_t)e.size(), e.data(), nullptr) == BP_EINVAL);
}

static void factor_graphs() {
    // triples along rows and columns plus diagonal pairs of an H x W grid
    for (int M : {3, 8, 33}) {
        const int H = 5, W = 6;
        std::vector<int32_t> fv, ft;
        for (int r = 0; r < H; ++r)
            for (int c = 0; c < W; ++c) {
                if (c + 2 < W) { fv.insert(fv.end(), {r * W + c, r * W + c + 1, r * W + c + 2}); ft.push_back(0); }
                if (r + 2 < H) { fv.insert(fv.end(), {r * W + c, (r + 1) * W + c, (r + 2) * W + c}); ft.push_back(1); }
                if (r + 1 < H && c + 1 < W) { fv.insert(fv.end(), {r * W + c, (r + 1) * W + c + 1, -1}); ft.push_back(2); }
            }
        std::vector<int32_t> t3, t2;
        std::vector<float> v3, v2;
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b) {
                if ((a + b) % 3 == 0) { t2.insert(t2.end(), {a, b}); v2.push_back(0.5f + 0.01f * a); }
                for (int c = 0; c < M; ++c)
                    if (a == b && b == c) { t3.insert(t3.end(), {a, b, c}); v3.push_back(1.0f); }
            }
        bp_factor_type types[3] = {{3, (int32_t)v3.size(), t3.data(), v3.data(), 0.1f},
                                   {3, (int32_t)v3.size(), t3.data(), v3.data(), 0.2f},
                                   {2, (int32_t)v2.size(), t2.data(), v2.data(), 0.05f}};
        bp_fgraph* F = nullptr;
        for (int dense : {0, 1})
            EXPECT(bp_fg_init(&F, H * W, M, (int32_t)ft.size(), fv.data(), ft.data(), 3, types, dense, nullptr) ==
                       BP_EHIP &&
                   F == nullptr);
        std::vector<int32_t> bad = fv;
        bad[1] = bad[0];  // repeated variable
        EXPECT(bp_fg_init(&F, H * W, M, (int32_t)ft.size(), bad.data(), ft.data(), 3, types, 0, nullptr) == BP_EINVAL);
        bad = fv;
        bad[4] = H * W;  // variable out of range
        EXPECT(bp_fg_init(&F, H * W, M, (int32_t)ft.size(), bad.data(), ft.data(), 3, types, 0, nullptr) == BP_EINVAL);
        std::vector<int32_t> badt = ft;
        badt[0] = 3;
        EXPECT(bp_fg_init(&F, H * W, M, (int32_t)ft.size(), fv.data(), badt.data(), 3, types, 0, nullptr) == BP_EINVAL);
        std::vector<int32_t> dup = t2;
        if (dup.size() >= 4) {
            dup[2] = dup[0];
            dup[3] = dup[1];
            bp_factor_type d2[3] = {types[0], types[1], {2, (int32_t)v2.size(), dup.data(), v2.data(), 0.05f}};
            EXPECT(bp_fg_init(&F, H * W, M, (int32_t)ft.size(), fv.data(), ft.data(), 3, d2, 0, nullptr) == BP_EINVAL);
        }
    }
}

static void noalloc_arguments() {
    float* g = static_cast<float*>(fake_device(1024));
    float* b = static_cast<float*>(fake_device(1024));
    EXPECT(bp_solve_noalloc(g, 4, 4, 4, 1, 1.0f, BP_FBAR_TIED, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC, nullptr, nullptr,
                            nullptr) == BP_EINVAL);
    EXPECT(bp_solve_noalloc(g, 0, 4, 4, 1, 1.0f, BP_FBAR_TIED, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC, b, nullptr, nullptr) ==
           BP_EINVAL);
    EXPECT(bp_solve_noalloc(g, 4, 4, 4, 1, 1.0f, BP_FBAR_TIED, BP_SUM_PRODUCT, 1, BP_SCHED_SYNC, b, nullptr, nullptr) ==
           BP_EHIP);
}

int main() {
    int n = 0;
    if (hipGetDeviceCount(&n) == hipSuccess && n > 0) {
        std::printf("a GPU is present: this check runs on machines without one\n");
        return 77;
    }
    null_handles();
    init_without_device();
    potentials_and_layouts();
    sparse_tables();
    batches();
    factor_graphs();
    noalloc_arguments();
    std::printf("host runtime: %d checks, %d failures\n", checks, failures);
    return failures ? 1 : 0;
}
