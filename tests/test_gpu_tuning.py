"""Launch mappings of the two-iteration launches (bp_set_launch_tuning,
bp_autotune): every mapping and workgroup cap computes the same messages
bit for bit, since all run the same per-pixel code; the autotuner keeps one
of them and resets the messages."""
import numpy as np
import pytest

from bp_gpu_util import say
from synth_mrf import random_unary

pytestmark = pytest.mark.gpu

LAYOUTS = ["strips", "wide", "bands", "slots", "walk", "tile"]
CAPS = [-1, 0, 4, 3, 2, 1]  # the walk ignores the cap (its LDS ring sets two workgroups per CU)
CASES = [  # H, W, M, T, alpha, mode, schedule, arith
    (37, 70, 64, 4, 0.5, "sum", "sync", "f64"),
    (37, 70, 64, 4, 0.5, "max", "sync", "f64"),
    (29, 51, 64, 4, 0.5, "sum", "checkerboard", "f64"),
    (40, 100, 16, 2, 1.0, "max", "checkerboard", "f64"),
    (30, 50, 48, 3, 0.7, "sum", "sync", "f64"),   # M not 4G: one group per slot whatever the layout
    (33, 90, 64, 4, 0.5, "sum", "sync", "f32"),
    (21, 34, 128, 6, 0.3, "sum", "sync", "f32"),
    # column walk (M = 32, 64; M = 128 runs the wide strips): strips of 256/G
    # columns (a ragged last strip), row chunks with halo rows, a single row,
    # and rows of missing senders at every border
    (5, 37, 32, 3, 0.8, "sum", "sync", "f64"),
    (1, 20, 64, 4, 0.5, "max", "sync", "f64"),
    (64, 16, 128, 8, 0.4, "max", "sync", "f64"),
    (300, 40, 64, 4, 0.5, "sum", "sync", "f32"),
    (97, 530, 32, 2, 1.1, "sum", "sync", "f32"),
    # the tile launch's checkerboard form: both colours' tile layouts, ragged
    # tiles, halo pixels of either colour at every border
    (37, 90, 32, 3, 0.6, "sum", "checkerboard", "f32"),
    (21, 45, 64, 4, 0.5, "max", "checkerboard", "f64"),
    (6, 9, 64, 4, 0.5, "sum", "checkerboard", "f32"),
    # tiles at M = 16 (8 x 8) and M = 128 (4 x 2, checkerboard 4 x 4)
    (45, 70, 16, 2, 1.0, "sum", "sync", "f32"),
    (19, 27, 16, 2, 1.0, "max", "sync", "f64"),
    (23, 37, 128, 8, 0.3, "sum", "checkerboard", "f32"),
]


def messages(grid, mode, schedule, n=6):
    import torch
    grid.reset()
    grid.iterate(mode, n, schedule)
    m = grid.get_messages().cpu().numpy()
    torch.cuda.synchronize()
    return m


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:4])) + f"_{c[5]}_{c[6]}_{c[7]}")
def test_every_mapping_gives_the_same_bits(case):
    import torch
    from paper_1010_0012_amd.grid import Grid
    H, W, M, T, alpha, mode, schedule, arith = case
    grid = Grid(H, W)
    grid.set_potential(M, T, alpha)
    grid.set_arithmetic(arith)
    grid.set_unary(torch.from_numpy(random_unary(H, W, M, 7 + M)).cuda())
    ref = messages(grid, mode, schedule)
    for layout in LAYOUTS:
        for cap in CAPS:
            say(f"{case}: layout {layout}, cap {cap}")
            grid.set_launch_tuning(layout, cap)
            assert grid.get_launch_tuning() == (layout, cap)
            np.testing.assert_array_equal(messages(grid, mode, schedule), ref)
    grid.set_launch_tuning("wide", -1)  # the autotuner starts from the current setting
    best = grid.autotune(mode, schedule, 2)
    layout, cap = grid.get_launch_tuning()
    say(f"{case}: autotuned {layout}, cap {cap}, {best:.1f} us per iteration")
    assert best > 0 and layout in LAYOUTS and cap in (-1, 0, 4, 3, 2)
    np.testing.assert_array_equal(messages(grid, mode, schedule), ref)
    grid.close()


def test_tuning_argument_errors():
    import torch
    from paper_1010_0012_amd import _lib as L
    from paper_1010_0012_amd.grid import Grid
    grid = Grid(8, 8)
    grid.set_potential(16, 2, 1.0)
    grid.set_unary(torch.from_numpy(random_unary(8, 8, 16, 1)).cuda())
    for layout, cap in ((6, -1), (-1, 0), (0, -2), (0, 65)):
        with pytest.raises(L.BPError) as e:
            L.bp_set_launch_tuning(grid.handle, layout, cap)
        assert e.value.status == L.BP_EINVAL
    for mode, schedule, trials in ((0, 0, 3), (0, 0, 0), (0, L.BP_SCHED_SWEEP, 2), (5, 0, 2)):
        with pytest.raises(L.BPError) as e:
            L.bp_autotune(grid.handle, mode, schedule, trials)
        assert e.value.status == L.BP_EINVAL
    assert grid.get_launch_tuning() == ("wide", -1)
    torch.cuda.synchronize()
    grid.close()


@pytest.mark.parametrize("layout", ["walk", "tile"])
@pytest.mark.parametrize("M,T,arith", [(32, 3, "f32"), (64, 4, "f64")])
def test_multiscale_same_bits_under_the_walk(M, T, arith, layout):
    """Multi-scale BP runs every level's synchronous pairs in the grid's
    mapping: the walk and the tile launch (coarse levels included) give the
    wide strips' bits."""
    import torch
    from paper_1010_0012_amd.grid import Grid
    H, W = 100, 130
    g = torch.from_numpy(random_unary(H, W, M, 11)).cuda()
    out = {}
    for lay in ("wide", layout):
        grid = Grid(H, W)
        grid.set_potential(M, T, 0.6)
        grid.set_arithmetic(arith)
        grid.set_unary(g)
        grid.set_launch_tuning(lay, -1)
        grid.iterate_multiscale("sum", (4, 6, 6))
        out[lay] = grid.get_messages().cpu().numpy()
        torch.cuda.synchronize()
        grid.close()
    np.testing.assert_array_equal(out[layout], out["wide"])
