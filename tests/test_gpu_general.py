"""GPU parity of general sparse-compatible potentials (Sec. 4 / Sec. 7) and of
the Eq. 10 max-product update, through the C ABI, against the oracle's
per-edge potentials (Eq. 7 for sum; Eq. 10, the split form, for max, which
is exact for any fbar).  Same bar as the other tests (bp_gpu_util.check)."""
import numpy as np
import pytest

from bp_gpu_util import check, run_oracle, say
from oracle import grid_bp as gb
from synth_mrf import random_unary

pytestmark = pytest.mark.gpu


def random_type(rng, M, density, below_fbar):
    """A random sparse-compatible potential (not a function of x - y), as
    (CSR over the second node's label, oracle Potential), float32 values."""
    fbar = np.float32(rng.uniform(0.05, 0.4))
    compat = rng.random((M, M)) < density
    compat[rng.permutation(M), np.arange(M)] = True   # every y has a compatible x
    lo = 0.0 if below_fbar else float(fbar)
    vals = rng.uniform(lo, lo + 1.0, (M, M)).astype(np.float32)
    col_ptr, row_idx, val = [0], [], []
    for y in range(M):
        xs = np.nonzero(compat[:, y])[0]
        row_idx += xs.tolist()
        val += vals[xs, y].tolist()
        col_ptr.append(len(row_idx))
    F = np.where(compat, vals.astype(np.float64), float(fbar))
    pot = gb.Potential(F, compat, float(fbar))
    return (np.array(col_ptr), np.array(row_idx), np.array(val, dtype=np.float32), float(fbar)), pot


def window_csr(M, T, alpha, fbar):
    """The truncated-linear potential as a CSR type (float32 table values)."""
    a32 = float(np.float32(alpha))
    col_ptr, row_idx, val = [0], [], []
    for y in range(M):
        for x in range(max(0, y - T), min(M - 1, y + T) + 1):
            row_idx.append(x)
            val.append(np.float32(np.exp(-a32 * abs(x - y))))
        col_ptr.append(len(row_idx))
    return np.array(col_ptr), np.array(row_idx), np.array(val, dtype=np.float32), float(fbar)


def run_general(g32, csr_types, th, tv, mode, schedule, n):
    import torch
    from paper_1010_0012_amd.grid import Grid
    H, W, M = g32.shape
    grid = Grid(H, W)
    grid.set_potential(M, 0, 1.0)
    th_t = None if th is None else torch.from_numpy(np.ascontiguousarray(th, dtype=np.uint8)).cuda()
    tv_t = None if tv is None else torch.from_numpy(np.ascontiguousarray(tv, dtype=np.uint8)).cuda()
    grid.set_sparse_potentials(csr_types, th_t, tv_t)
    grid.set_unary(torch.from_numpy(np.ascontiguousarray(g32)).cuda())
    grid.iterate(mode, n, schedule)
    out = grid.get_messages().cpu().numpy(), grid.beliefs().cpu().numpy(), grid.map_labels().cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    return out


# (H, W, M, n_types, density): every lane class, ragged rows, one to four types
CASES = [(5, 7, 5, 1, 0.4), (6, 5, 16, 3, 0.2), (4, 6, 32, 2, 0.1), (3, 5, 64, 4, 0.08),
         (3, 4, 100, 2, 0.05), (3, 4, 128, 3, 0.05), (2, 3, 200, 2, 0.03), (2, 2, 256, 1, 0.03),
         (1, 9, 12, 2, 0.3), (9, 1, 12, 2, 0.3), (17, 13, 16, 4, 0.2)]


def _id(c):
    return "H{}W{}M{}K{}".format(*c[:4])


@pytest.mark.parametrize("schedule", ["sync", "checkerboard", "sweep"])
@pytest.mark.parametrize("mode,below", [("sum", False), ("sum", True), ("max", False), ("max", True)])
@pytest.mark.parametrize("case", CASES, ids=_id)
def test_general_potentials(case, mode, below, schedule):
    H, W, M, K, density = case
    rng = np.random.default_rng(1000 + CASES.index(case))
    pairs = [random_type(rng, M, density, below) for _ in range(K)]
    th = rng.integers(0, K, (H, W - 1))
    tv = rng.integers(0, K, (H - 1, W))
    pot = gb.EdgePotentials([p for _, p in pairs], th, tv)
    g32 = random_unary(H, W, M, 2000 + CASES.index(case))
    n = {"sync": 4, "checkerboard": 6, "sweep": 2}[schedule]
    tag = f"general {mode} below={below} {schedule} {_id(case)}"
    say(tag)
    gpu = run_general(g32, [c for c, _ in pairs], th, tv, mode, schedule, n)
    impl = gb.SPARSE if mode == "sum" else gb.SPLIT   # Eq. 7; Eq. 10 (exact for any fbar)
    check(tag, gpu, g32, M, 0, 1.0, None, mode, schedule, n, impl, pot=pot)


@pytest.mark.parametrize("schedule", ["sync", "checkerboard", "sweep"])
@pytest.mark.parametrize("M,T,alpha", [(16, 2, 1.0), (64, 4, 0.5), (128, 8, 0.3), (20, 5, 0.6), (200, 10, 0.2),
                                       (64, 20, 0.1)])
def test_window_max_eq10(M, T, alpha, schedule):
    """Truncated-linear max-product with fbar above f(T): Eq. 11 would be
    wrong, the library runs Eq. 10 (the window kernels' prefix/suffix-max
    form, or the general kernel beyond the register windows, T = 20); equal
    to the oracle's Eq. 10 and, bit for bit, to the dense Eq. 9 kernel."""
    from bp_gpu_util import run_gpu
    H, W = 6, 7
    g32 = random_unary(H, W, M, 3000 + M)
    fbar = float(np.float32(np.exp(-alpha * T) * 1.5 + 0.01))
    n = {"sync": 5, "checkerboard": 6, "sweep": 2}[schedule]
    say(f"window max Eq. 10 {schedule} M={M} T={T} fbar={fbar:.4f}")
    gs = run_gpu(g32, M, T, alpha, fbar, "max", schedule, n)
    check(f"window Eq. 10 {schedule} M={M}", gs, g32, M, T, alpha, fbar, "max", schedule, n, gb.SPLIT)
    if M <= 128:
        gd = run_gpu(g32, M, T, alpha, fbar, "max", schedule, n, dense=True)
        np.testing.assert_array_equal(gs[0], gd[0])
        np.testing.assert_array_equal(gs[1], gd[1])


@pytest.mark.parametrize("M,T", [(16, 2), (64, 4), (128, 8)])
def test_window_as_csr_matches_window_kernel_max(M, T):
    """The truncated-linear potential given as a CSR type runs the same
    float32 products as the window kernel: max-product results are equal bit
    for bit."""
    from bp_gpu_util import run_gpu
    H, W, alpha = 5, 6, 0.7
    g32 = random_unary(H, W, M, 4000 + M)
    fbar = float(np.float32(np.exp(-float(np.float32(alpha)) * T)))
    a = run_gpu(g32, M, T, alpha, fbar, "max", "sync", 4)
    b = run_general(g32, [window_csr(M, T, alpha, fbar)], None, None, "max", "sync", 4)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_general_errors():
    import torch
    from paper_1010_0012_amd import _lib as L
    h = L.bp_init_grid(4, 5)
    L.bp_set_potential(h, 8, 2, 1.0, L.BP_FBAR_TIED)
    nbytes = L.bp_workspace_bytes(h)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L.bp_attach_workspace(h, ws, nbytes)
    L.bp_set_unary(h, torch.rand(4, 5, 8, device="cuda") + 0.1)
    good = window_csr(8, 2, 1.0, 0.1)
    cp, ri, va, fb = good
    bad_cases = [
        [(cp, ri[::-1].copy(), va, fb)],                        # labels not increasing
        [(cp, np.where(ri == 0, 9, ri), va, fb)],              # label out of range
        [(cp, ri, -va, fb)],                                   # negative value
        [(cp, ri, va, -1.0)],                                  # negative fbar
        [(np.concatenate([[1], cp[1:]]), ri, va, fb)],         # col_ptr[0] != 0
    ]
    for types in bad_cases:
        with pytest.raises(L.BPError) as e:
            L.bp_sparse_table_bytes(h, types)
        assert e.value.status == L.BP_EINVAL
    with pytest.raises(L.BPError) as e:
        L.bp_sparse_table_bytes(h, [good] * 17)
    assert e.value.status == L.BP_EINVAL
    tb = L.bp_sparse_table_bytes(h, [good, good])
    tab = torch.empty(tb, dtype=torch.uint8, device="cuda")
    th_bad = torch.full((4, 4), 2, dtype=torch.uint8, device="cuda")      # type 2 of 2
    with pytest.raises(L.BPError) as e:
        L.bp_set_sparse_potentials(h, [good, good], tab, tb, th_bad, None)
    assert e.value.status == L.BP_EINVAL
    with pytest.raises(L.BPError) as e:
        L.bp_set_sparse_potentials(h, [good, good], tab, tb - 1, None, None)
    assert e.value.status == L.BP_ENOMEM
    L.bp_set_sparse_potentials(h, [good, good], tab, tb, None, None)
    L.bp_iterate(h, L.BP_SUM_PRODUCT, 2, L.BP_SCHED_SYNC)
    L.bp_iterate(h, L.BP_MAX_PRODUCT, 2, L.BP_SCHED_CHECKERBOARD)
    L.bp_iterate(h, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SWEEP)
    with pytest.raises(L.BPError) as e:
        L.bp_iterate_dense(h, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SYNC)
    assert e.value.status == L.BP_EUNSUPPORTED
    L.bp_set_potential(h, 8, 2, 1.0, L.BP_FBAR_TIED)                      # back to the window
    L.bp_iterate_dense(h, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SYNC)
    torch.cuda.synchronize()
    L.bp_destroy(h)


def test_general_full_size_sampled():
    """480 x 640, M = 64, four per-edge types, 20 sum-product iterations: every
    sampled message of the last step equals the oracle's update of the GPU's
    previous state (<= 1e-6); message sums within 1e-5 of 1."""
    import torch
    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import CONFIGS, make_config
    cfg = CONFIGS["stereo480x640"]
    g32, _ = make_config(cfg)
    H, W, M = g32.shape
    rng = np.random.default_rng(5000)
    pairs = [random_type(rng, M, 0.1, False) for _ in range(4)]
    th = rng.integers(0, 4, (H, W - 1))
    tv = rng.integers(0, 4, (H - 1, W))
    pot = gb.EdgePotentials([p for _, p in pairs], th, tv)
    grid = Grid(H, W)
    grid.set_potential(M, 0, 1.0)
    grid.set_sparse_potentials([c for c, _ in pairs], torch.from_numpy(th.astype(np.uint8)).cuda(),
                               torch.from_numpy(tv.astype(np.uint8)).cuda())
    grid.set_unary(torch.from_numpy(g32).cuda())
    say("general 480x640 M=64 four types x20")
    grid.iterate("sum", 19)
    prev = grid.get_messages().cpu().numpy().astype(np.float64)
    grid.iterate("sum", 1)
    last = grid.get_messages().cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    g64 = g32.astype(np.float64)
    worst, checked = 0.0, 0
    while checked < 120:
        r, c, o = int(rng.integers(0, H)), int(rng.integers(0, W)), int(rng.integers(0, 4))
        dr, dc = gb.OFFSETS[o]
        if not (0 <= r + dr < H and 0 <= c + dc < W):
            continue
        want = gb.single_update(g64, prev, pot, "sum", r, c, o)
        worst = max(worst, float(np.max(np.abs(last[gb.OPPOSITE[o], r + dr, c + dc] - want))))
        checked += 1
    sums = gb.message_sums(last)
    say(f"general full size: sampled max|dm| = {worst:.2e}, |sum - 1| <= {np.max(np.abs(sums - 1)):.2e}")
    assert worst <= 1e-6
    assert np.max(np.abs(sums - 1.0)) <= 1e-5


@pytest.mark.parametrize("schedule", ["sync", "checkerboard"])
def test_general_offsets_beyond_2_31(schedule):
    """A 4096 x 4096 grid with M = 40 (message buffers beyond 2^31 floats):
    the general kernel on the truncated-linear potential as a CSR type equals
    the window kernel bit for bit (max-product), over the whole buffer."""
    import torch
    from paper_1010_0012_amd.grid import Grid
    H = W = 4096
    M, T, alpha = 40, 3, 0.7
    say(f"general offsets beyond 2^31: {H}x{W}x{M} {schedule}")
    gen = torch.Generator(device="cuda").manual_seed(41)
    g = torch.rand((H, W, M), generator=gen, device="cuda") * 0.9 + 0.1
    fbar = float(np.float32(np.exp(-float(np.float32(alpha)) * T)))
    grid = Grid(H, W)
    grid.set_potential(M, T, alpha, fbar)
    grid.set_unary(g)
    grid.iterate("max", 2, schedule)
    window = grid.get_messages()
    grid.set_sparse_potentials([window_csr(M, T, alpha, fbar)])
    grid.reset()
    grid.iterate("max", 2, schedule)
    torch.cuda.synchronize()
    assert 4 * H * W * M > 2 ** 31
    assert torch.equal(grid.get_messages(), window)
    grid.close()
