"""bp_solve_noalloc (the entry point that allocates nothing) against the
handle calls it stands for (bp_init_grid, bp_set_potential, workspace,
bp_set_unary, bp_iterate, bp_readout): the same beliefs and labels bit for
bit, on two calls in a row, the second on a smaller grid, so that the
second call runs over the first call's leftovers in the shared array."""
import numpy as np
import pytest

from bp_gpu_util import say
from synth_mrf import random_unary

pytestmark = pytest.mark.gpu

# (H, W, M, T, alpha, fbar, mode, schedule, n): a larger call, then a smaller one
PAIRS = [
    [(96, 120, 64, 4, 0.5, None, "sum", "sync", 7), (33, 17, 16, 2, 1.0, None, "sum", "sync", 6)],
    [(64, 80, 32, 3, 0.7, None, "max", "checkerboard", 9), (5, 7, 20, 3, 0.6, None, "max", "checkerboard", 4)],
    [(256, 256, 32, 3, 1.0, None, "sum", "sync", 5), (40, 50, 128, 8, 0.3, 0.0, "sum", "sweep", 2)],
]


def handle_solve(g, H, W, M, T, alpha, fbar, mode, schedule, n):
    import torch
    from paper_1010_0012_amd.grid import Grid
    grid = Grid(H, W)
    grid.set_potential(M, T, alpha, fbar)
    grid.set_unary(g)
    grid.iterate(mode, n, schedule)
    b = torch.empty((H, W, M), dtype=torch.float32, device="cuda")
    lab = torch.empty((H, W), dtype=torch.int32, device="cuda")
    grid.readout(b, lab)
    out = b.cpu().numpy(), lab.cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    return out


@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: "{}x{}x{}_then_{}x{}x{}".format(*p[0][:3], *p[1][:3]))
def test_noalloc_equals_handle_calls(pair):
    import torch
    from paper_1010_0012_amd import _lib as L
    for k, (H, W, M, T, alpha, fbar, mode, schedule, n) in enumerate(pair):
        say(f"noalloc call {k}: {H}x{W}x{M} T={T} {mode} {schedule} x{n}")
        g = torch.from_numpy(random_unary(H, W, M, 900 + 10 * k + M)).cuda()
        b = torch.full((H, W, M), -1.0, dtype=torch.float32, device="cuda")
        lab = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
        L.bp_solve_noalloc(g, H, W, M, T, alpha, fbar, getattr(L, f"BP_{mode.upper()}_PRODUCT"), n,
                           getattr(L, f"BP_SCHED_{schedule.upper()}"), b, lab)
        got_b, got_l = b.cpu().numpy(), lab.cpu().numpy()
        torch.cuda.synchronize()
        want_b, want_l = handle_solve(g, H, W, M, T, alpha, fbar, mode, schedule, n)
        np.testing.assert_array_equal(got_b, want_b)
        np.testing.assert_array_equal(got_l, want_l)


def test_noalloc_rejects_oversize_and_bad_arguments():
    import torch
    from paper_1010_0012_amd import _lib as L
    g = torch.ones(8, dtype=torch.float32, device="cuda")
    b = torch.empty(8, dtype=torch.float32, device="cuda")
    with pytest.raises(L.BPError) as e:          # 300 x 300 x 64 needs far more than the fixed array
        L.bp_solve_noalloc(g, 300, 300, 64, 4, 0.5, None, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SYNC, b, None)
    assert e.value.status == L.BP_EINVAL
    with pytest.raises(L.BPError) as e:          # no output
        L.bp_solve_noalloc(g, 2, 2, 2, 1, 0.5, None, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SYNC, None, None)
    assert e.value.status == L.BP_EINVAL
    with pytest.raises(L.BPError) as e:          # T >= M
        L.bp_solve_noalloc(g, 2, 2, 2, 2, 0.5, None, L.BP_SUM_PRODUCT, 1, L.BP_SCHED_SYNC, b, None)
    assert e.value.status == L.BP_EINVAL
    torch.cuda.synchronize()
