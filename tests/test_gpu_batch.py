"""Batched path: many grids of uneven H x W, M, T, alpha in one persistent
launch per iteration, replayed from HIP graphs.

Every instance must equal a single-grid run of the same problem bit for bit
(the batched kernel runs the same arithmetic; wider windows only add taps of
weight 0, which add exact zeros) and match the FP64 oracle to the parity bar.
"""
import numpy as np
import pytest

from bp_gpu_util import check, compare, run_gpu, run_oracle, say
from oracle import grid_bp as gb
from synth_mrf import make_batch_configs, make_batch_instance, random_unary

pytestmark = pytest.mark.gpu

SMALL = [  # H, W, M, T, alpha, fbar
    (9, 13, 16, 2, 1.0, None),
    (7, 5, 5, 1, 0.8, None),
    (6, 11, 20, 3, 0.6, None),
    (5, 8, 32, 8, 0.4, None),
    (4, 6, 64, 4, 0.5, None),
    (3, 7, 100, 6, 0.3, None),
    (3, 5, 128, 8, 0.2, None),
    (1, 9, 12, 0, 1.0, 0.3),
    (8, 1, 16, 5, 0.7, 0.01),
    (2, 3, 48, 7, 0.9, None),
]


def make_batch(specs, seeds, graphs=True):
    import torch
    from paper_1010_0012_amd.batch import Batch
    gs = [torch.from_numpy(random_unary(H, W, M, s)).cuda() for (H, W, M, *_), s in zip(specs, seeds)]
    grids = [(g, T, a, f) for g, (H, W, M, T, a, f) in zip(gs, specs)]
    return Batch(grids, graphs=graphs), gs


def results(batch):
    import torch
    b = [x.cpu().numpy() for x in batch.beliefs()]
    lab = [x.cpu().numpy() for x in batch.map_labels()]
    torch.cuda.synchronize()
    return b, lab


@pytest.mark.parametrize("mode", ["sum", "max"])
def test_small_batch_matches_single_and_oracle(mode):
    seeds = list(range(len(SMALL)))
    batch, gs = make_batch(SMALL, seeds)
    n = 6
    say(f"batch {mode} x{n}: {len(SMALL)} instances")
    batch.iterate(mode, n)
    bb, bl = results(batch)
    for j, (H, W, M, T, a, f) in enumerate(SMALL):
        g32 = gs[j].cpu().numpy()
        _, b1, l1 = run_gpu(g32, M, T, a, f, mode, "sync", n, want_messages=False)
        np.testing.assert_array_equal(bb[j], b1)
        np.testing.assert_array_equal(bl[j], l1)
        check(f"batch[{j}] {mode}", (None, bb[j], bl[j]), g32, M, T, a, f, mode, "sync", n, check_msgs=False)
    batch.close()


def test_graph_replays_match_eager():
    """Replays of a captured graph, with eager work and synchronisation between
    them, equal direct launches after every replay."""
    import torch
    seeds = [100 + i for i in range(len(SMALL))]
    bg, _ = make_batch(SMALL, seeds, graphs=True)
    be, _ = make_batch(SMALL, seeds, graphs=False)
    for rep in range(4):
        bg.iterate("sum", 3)
        be.iterate("sum", 3)
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # unrelated eager work between replays
        torch.cuda.synchronize()
        del junk
        rg, re_ = results(bg), results(be)
        for x, y in zip(rg[0] + rg[1], re_[0] + re_[1]):
            np.testing.assert_array_equal(x, y)
    # odd iteration counts flip the buffer parity: both parities are captured
    bg.iterate("sum", 1)
    be.iterate("sum", 1)
    bg.iterate("max", 2)
    be.iterate("max", 2)
    rg, re_ = results(bg), results(be)
    for x, y in zip(rg[0] + rg[1], re_[0] + re_[1]):
        np.testing.assert_array_equal(x, y)
    bg.close()
    be.close()


def test_plans_do_not_change_results():
    seeds = [200 + i for i in range(len(SMALL))]
    batch, _ = make_batch(SMALL, seeds)
    batch.iterate("sum", 4)
    ref = results(batch)
    for streams, passes, grid in ((4, [1, 1, 1, 1, 1], 1), (1, [3, 5, 2, 7, 1], 7), (2, [64, 32, 16, 16, 4], 1024),
                                  (1, [2, 2, 2, 2, 2], 1 << 30), (1, [1, 1, 1, 1, 1], 1 << 30)):
        batch.set_streams(streams)
        batch.set_plan(passes, grid)
        batch.reset()
        batch.iterate("sum", 4)
        got = results(batch)
        for x, y in zip(got[0] + got[1], ref[0] + ref[1]):
            np.testing.assert_array_equal(x, y)
    best = batch.autotune("sum", 2)
    plan = batch.get_plan()
    say(f"autotuned plan {plan}, {batch.get_streams()} streams, {best:.1f} us/iteration")
    batch.iterate("sum", 4)
    got = results(batch)
    for x, y in zip(got[0] + got[1], ref[0] + ref[1]):
        np.testing.assert_array_equal(x, y)
    batch.close()


def test_batch_errors():
    import torch
    from paper_1010_0012_amd import _lib as L
    g = torch.rand(4, 4, 16, device="cuda") + 0.1
    with pytest.raises(L.BPError) as e:
        L.bp_batch_init([L.bp_grid_desc(4, 4, 16, 9, 1.0, L.BP_FBAR_TIED, g.data_ptr())])
    assert e.value.status == L.BP_EUNSUPPORTED  # T > 8
    with pytest.raises(L.BPError) as e:
        L.bp_batch_init([L.bp_grid_desc(4, 4, 16, 2, 1.0, -3.0, g.data_ptr())])
    assert e.value.status == L.BP_EINVAL
    h = L.bp_batch_init([L.bp_grid_desc(4, 4, 16, 2, 1.0, 0.5, g.data_ptr())])
    with pytest.raises(L.BPError) as e:
        L.bp_batch_iterate(h, 0, 1)                    # no workspace
    assert e.value.status == L.BP_ESTATE
    nbytes = L.bp_batch_workspace_bytes(h)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L.bp_batch_attach_workspace(h, ws, nbytes)
    with pytest.raises(L.BPError) as e:
        L.bp_batch_iterate(h, 1, 1)                    # fbar 0.5 > f(2): no max-product
    assert e.value.status == L.BP_EUNSUPPORTED
    torch.cuda.synchronize()
    L.bp_batch_destroy(h)


def test_batch32_full():
    """The 32-instance workload (H, W in [64, 512], M in {16,...,128}, T in
    [1, 8]), 30 sum-product iterations: every instance bitwise equal to its
    single-grid run, which the single-grid tests tie to the oracle; the two
    smallest instances are also compared with the oracle directly."""
    import torch
    from paper_1010_0012_amd.batch import Batch
    insts = make_batch_configs()
    data = [make_batch_instance(i) for i in insts]
    gs = [torch.from_numpy(g).cuda() for g, _ in data]
    batch = Batch([(g, i.T, i.alpha) for g, i in zip(gs, insts)])
    n = 30
    say(f"batch32 sum x{n}")
    batch.iterate("sum", n)
    bb, bl = results(batch)
    for j, it in enumerate(insts):
        _, b1, l1 = run_gpu(data[j][0], it.M, it.T, it.alpha, None, "sum", "sync", n, want_messages=False)
        np.testing.assert_array_equal(bb[j], b1)
        np.testing.assert_array_equal(bl[j], l1)
    small = sorted(range(len(insts)), key=lambda j: insts[j].H * insts[j].W * insts[j].M)[:2]
    for j in small:
        it = insts[j]
        compare(f"batch32[{j}] {it.H}x{it.W} M={it.M} T={it.T}", (None, bb[j], bl[j]),
                run_oracle(data[j][0], it.M, it.T, it.alpha, None, "sum", "sync", n, gb.DENSE),
                check_msgs=False)
    batch.close()


# Instances for the float32 setting: every lane class with M = 4G (float32
# where fbar > 0), one M that is not 4G and one fbar = 0 instance in a code
# path of its own (both stay in double, as a single grid does), and a grid
# wide and tall enough for interior waves in the row-block launch.
F32_SPECS = [  # H, W, M, T, alpha, fbar
    (9, 13, 16, 2, 1.0, None),
    (8, 1, 16, 5, 0.7, 0.01),
    (6, 11, 20, 3, 0.6, None),
    (5, 8, 32, 8, 0.4, None),
    (20, 70, 32, 2, 0.7, None),
    (4, 6, 64, 4, 0.5, None),
    (12, 40, 64, 4, 0.8, None),
    (7, 9, 64, 3, 0.5, 0.0),
    (3, 5, 128, 8, 0.2, None),
]


@pytest.mark.parametrize("n", [6, 5])
def test_f32_batch_equals_single_grids(n):
    """With float32 arithmetic every instance equals its single-grid solve
    with float32 arithmetic bit for bit (instances without a float32 kernel
    run in double on both sides), under the row-block launches and under a
    persistent plan; the wide instance really ran in float32 (it differs
    from the double batch)."""
    seeds = [300 + i for i in range(len(F32_SPECS))]
    batch, gs = make_batch(F32_SPECS, seeds)
    batch.set_arithmetic("f32")
    say(f"batch f32 sum x{n}: {len(F32_SPECS)} instances")
    batch.iterate("sum", n)
    bb, bl = results(batch)
    for j, (H, W, M, T, a, f) in enumerate(F32_SPECS):
        _, b1, l1 = run_gpu(gs[j].cpu().numpy(), M, T, a, f, "sum", "sync", n, want_messages=False, arith="f32")
        np.testing.assert_array_equal(bb[j], b1, err_msg=f"instance {j}")
        np.testing.assert_array_equal(bl[j], l1, err_msg=f"instance {j}")
    batch.set_plan([2, 2, 2, 2, 2], 7)  # persistent: no row-block layout
    batch.reset()
    batch.iterate("sum", n)
    got = results(batch)
    for x, y in zip(got[0] + got[1], bb + bl):
        np.testing.assert_array_equal(x, y)
    batch.set_arithmetic("f64")
    batch.reset()
    batch.iterate("sum", n)
    b64, _ = results(batch)
    assert not np.array_equal(b64[4], bb[4])
    np.testing.assert_allclose(b64[4], bb[4], rtol=0, atol=1e-5)
    batch.close()
