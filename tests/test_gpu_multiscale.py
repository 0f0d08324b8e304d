"""GPU parity of coarse-to-fine (multi-scale) BP against the oracle's
multiscale.run, FP64 and float32-storage model (bp_gpu_util.check_against),
and a full-size sampled check in the benchmark's configuration."""
import numpy as np
import pytest

from bp_gpu_util import check_against, library_potential, oracle_result, say
from oracle import grid_bp as gb
from oracle import multiscale as ms
from synth_mrf import CONFIGS, make_config, random_unary

pytestmark = pytest.mark.gpu


def run_ms(g32, M, T, alpha, mode, iters, fbar=None, csr_types=None, type_maps=None):
    import torch
    from paper_1010_0012_amd.grid import Grid
    H, W, _ = g32.shape
    grid = Grid(H, W)
    grid.set_potential(M, T, alpha, fbar)
    if csr_types is not None:
        grid.set_sparse_potentials(csr_types, *(type_maps or (None, None)))
    grid.set_unary(torch.from_numpy(np.ascontiguousarray(g32)).cuda())
    grid.iterate_multiscale(mode, iters)
    out = grid.get_messages().cpu().numpy(), grid.beliefs().cpu().numpy(), grid.map_labels().cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    return out


# (H, W, M, T, alpha, iters): odd sizes (partial blocks), every lane class,
# one to four coarser levels, zero iterations at some levels
CASES = [(5, 7, 5, 1, 0.8, [3, 3]), (9, 11, 16, 2, 1.0, [2, 3, 4]), (16, 16, 32, 3, 0.7, [3, 0, 5]),
         (13, 10, 64, 4, 0.5, [2, 2, 2, 2]), (7, 6, 128, 8, 0.3, [2, 3]), (6, 5, 200, 10, 0.3, [1, 2]),
         (33, 17, 16, 2, 1.0, [2, 2, 2, 2, 3]), (1, 9, 8, 1, 1.0, [3, 3]), (4, 4, 12, 2, 0.9, [0, 4])]


def _id(c):
    return "H{}W{}M{}T{}L{}".format(c[0], c[1], c[2], c[3], len(c[5]) - 1)


@pytest.mark.parametrize("mode", ["sum", "max"])
@pytest.mark.parametrize("case", CASES, ids=_id)
def test_multiscale(case, mode):
    H, W, M, T, alpha, iters = case
    g32 = random_unary(H, W, M, 6000 + CASES.index(case))
    tag = f"multiscale {mode} {_id(case)} iters={iters}"
    say(tag)
    gpu = run_ms(g32, M, T, alpha, mode, iters)
    pot = library_potential(M, T, alpha, None, mode)
    g = g32.astype(np.float64)
    levels = len(iters) - 1
    ref = oracle_result(g32, ms.run(g, pot, mode, levels, iters))
    ref32 = oracle_result(g32, ms.run(g, pot, mode, levels, iters, storage=np.float32))
    check_against(tag, gpu, g32, ref, ref32)


# (H, W, M, T, alpha, fbar, iters): fbar above f(T), so max-product needs Eq. 10
EQ10_CASES = [(9, 11, 16, 2, 1.0, 0.3, [2, 3, 4]), (13, 10, 64, 4, 0.5, 0.5, [2, 2, 2, 2]),
              (7, 6, 128, 8, 0.3, 0.2, [2, 3]), (6, 5, 200, 10, 0.3, 0.1, [1, 2])]


@pytest.mark.parametrize("case", EQ10_CASES, ids=lambda c: _id(c[:5] + c[6:]))
def test_multiscale_eq10(case):
    """Max-product with fbar above f(T): every level runs Eq. 10."""
    H, W, M, T, alpha, fbar, iters = case
    g32 = random_unary(H, W, M, 6100 + EQ10_CASES.index(case))
    tag = f"multiscale max Eq. 10 {_id(case[:5] + case[6:])} fbar={fbar}"
    say(tag)
    gpu = run_ms(g32, M, T, alpha, "max", iters, fbar=fbar)
    pot = library_potential(M, T, alpha, fbar, "max")
    g = g32.astype(np.float64)
    levels = len(iters) - 1
    ref = oracle_result(g32, ms.run(g, pot, "max", levels, iters, impl=gb.SPLIT))
    ref32 = oracle_result(g32, ms.run(g, pot, "max", levels, iters, impl=gb.SPLIT, storage=np.float32))
    check_against(tag, gpu, g32, ref, ref32)


@pytest.mark.parametrize("mode,below", [("sum", False), ("sum", True), ("max", False), ("max", True)])
@pytest.mark.parametrize("case", [(9, 11, 16, 0.2, [2, 3, 4]), (6, 7, 64, 0.08, [2, 2, 3])],
                         ids=lambda c: "H{}W{}M{}".format(*c[:3]))
def test_multiscale_general_potential(case, mode, below):
    """One general sparse-compatible potential on every edge (no type maps):
    Eq. 7 (sum), Eq. 11 or Eq. 10 (max) at every level."""
    from test_gpu_general import random_type
    H, W, M, density, iters = case
    rng = np.random.default_rng(6200 + M)
    csr, pot = random_type(rng, M, density, below)
    g32 = random_unary(H, W, M, 6300 + M)
    tag = f"multiscale general {mode} below={below} H{H}W{W}M{M}"
    say(tag)
    gpu = run_ms(g32, M, 0, 1.0, mode, iters, csr_types=[csr])
    impl = gb.SPARSE if mode == "sum" else gb.SPLIT
    g = g32.astype(np.float64)
    levels = len(iters) - 1
    ref = oracle_result(g32, ms.run(g, pot, mode, levels, iters, impl=impl))
    ref32 = oracle_result(g32, ms.run(g, pot, mode, levels, iters, impl=impl, storage=np.float32))
    check_against(tag, gpu, g32, ref, ref32)


def test_zero_levels_is_fresh_plain_solve():
    from bp_gpu_util import run_gpu
    g32 = random_unary(8, 9, 16, 77)
    a = run_ms(g32, 16, 2, 1.0, "sum", [6])
    b = run_gpu(g32, 16, 2, 1.0, None, "sum", "sync", 6)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("mode", ["sum", "max"])
def test_multiscale_pairs_equal_single_launches(mode):
    """Levels run two synchronous iterations per launch; the result equals
    single launches bit for bit (odd and even counts per level)."""
    import torch
    from paper_1010_0012_amd.grid import Grid
    g32 = random_unary(37, 29, 32, 91)
    out = []
    for fuse in (True, False):
        grid = Grid(37, 29)
        grid.set_potential(32, 3, 0.7)
        grid.set_sync_fusion(fuse)
        grid.set_unary(torch.from_numpy(g32).cuda())
        grid.iterate_multiscale(mode, [5, 2, 3, 4])
        out.append(grid.get_messages().cpu().numpy())
        torch.cuda.synchronize()
        grid.close()
    np.testing.assert_array_equal(out[0], out[1])


def test_multiscale_full_size_sampled():
    """480 x 640, M = 64, three coarser levels: after the solve one more plain
    iteration; every sampled message equals the oracle's update of the GPU's
    state (<= 1e-6), message sums within 1e-5 of 1, beliefs by Eq. 3."""
    import torch
    from paper_1010_0012_amd.grid import Grid
    cfg = CONFIGS["stereo480x640"]
    g32, _ = make_config(cfg)
    H, W, M = g32.shape
    grid = Grid(H, W)
    grid.set_potential(M, cfg.T, cfg.alpha)
    grid.set_unary(torch.from_numpy(g32).cuda())
    say("multiscale 480x640 levels=3 iters [10, 10, 10, 10]")
    grid.iterate_multiscale("sum", [10, 10, 10, 10])
    prev = grid.get_messages().cpu().numpy().astype(np.float64)
    grid.iterate("sum", 1)
    last = grid.get_messages().cpu().numpy()
    b = grid.beliefs().cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    pot = gb.truncated_linear(M, cfg.T, float(np.float32(cfg.alpha)))
    g64 = g32.astype(np.float64)
    rng = np.random.default_rng(8)
    worst, checked = 0.0, 0
    while checked < 120:
        r, c, o = int(rng.integers(0, H)), int(rng.integers(0, W)), int(rng.integers(0, 4))
        dr, dc = gb.OFFSETS[o]
        if not (0 <= r + dr < H and 0 <= c + dc < W):
            continue
        want = gb.single_update(g64, prev, pot, "sum", r, c, o)
        worst = max(worst, float(np.max(np.abs(last[gb.OPPOSITE[o], r + dr, c + dc] - want))))
        worst = max(worst, float(np.max(np.abs(b[r, c] - gb.single_belief(g64, last.astype(np.float64), r, c)))))
        checked += 1
    sums = gb.message_sums(last)
    say(f"multiscale full size: sampled max|d| = {worst:.2e}, |sum - 1| <= {np.max(np.abs(sums - 1)):.2e}")
    assert worst <= 1e-6
    assert np.max(np.abs(sums - 1.0)) <= 1e-5


def test_multiscale_errors():
    import torch
    from paper_1010_0012_amd import _lib as L
    h = L.bp_init_grid(6, 6)
    L.bp_set_potential(h, 8, 2, 1.0, L.BP_FBAR_TIED)
    nbytes = L.bp_workspace_bytes(h)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L.bp_attach_workspace(h, ws, nbytes)
    L.bp_set_unary(h, torch.rand(6, 6, 8, device="cuda") + 0.1)
    mb = L.bp_multiscale_workspace_bytes(h, 2)
    mws = torch.empty(mb, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.BPError) as e:
        L.bp_iterate_multiscale(h, 0, [1, 1, 1], mws, mb - 1)
    assert e.value.status == L.BP_ENOMEM
    with pytest.raises(L.BPError) as e:
        L.bp_iterate_multiscale(h, 0, [1, -1, 1], mws, mb)
    assert e.value.status == L.BP_EINVAL
    with pytest.raises(L.BPError) as e:
        L.bp_multiscale_workspace_bytes(h, 13)
    assert e.value.status == L.BP_EINVAL
    L.bp_iterate_multiscale(h, 0, [1, 1, 1], mws, mb)
    L.bp_set_potential(h, 8, 2, 1.0, 0.9)                  # fbar above f(2): Eq. 10
    L.bp_iterate_multiscale(h, 1, [1, 1, 1], mws, mb)
    from test_gpu_general import window_csr
    tb = L.bp_sparse_table_bytes(h, [window_csr(8, 2, 1.0, 0.1)] * 2)
    tabs = torch.empty(tb, dtype=torch.uint8, device="cuda")
    th = torch.zeros(6, 5, dtype=torch.uint8, device="cuda")
    tv = torch.ones(5, 6, dtype=torch.uint8, device="cuda")
    L.bp_set_sparse_potentials(h, [window_csr(8, 2, 1.0, 0.1)] * 2, tabs, tb, th, tv)
    with pytest.raises(L.BPError) as e:                    # type maps: finest level only
        L.bp_iterate_multiscale(h, 0, [1, 1, 1], mws, mb)
    assert e.value.status == L.BP_EUNSUPPORTED
    torch.cuda.synchronize()
    L.bp_destroy(h)
