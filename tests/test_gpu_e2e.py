"""End-to-end parity at full size: whole GPU solves of the benchmark-sized
workloads against the FP64 oracle's own whole solves.

The references (tests/golden/e2e_*.npz) are written by
tests/golden/make_e2e_ref.py, which runs only the oracle: the MAP labels and
top-two margins of every pixel, and FP64 beliefs at a fixed sample of 4096
pixels (corners, borders, the lowest margins, the pixels where float32
storage moves the result most, and uniform ones).  The GPU runs each
workload from the uniform start in the launch configuration the benchmark
times (two synchronous iterations or two checkerboard passes per launch; the
32-grid batch for the batched instance), then reads beliefs and labels (Eq. 3,
Sec. 6 disparity map).

Bar: beliefs within 1e-5 of FP64 on the sample, MAP labels equal wherever
the FP64 top-two margin exceeds 1e-6.  A case where the oracle's own
float32-storage model misses that bar must be named in STORAGE_LIMITED; it
is then held to the storage model instead (beliefs within 1e-6, labels equal
where its margin exceeds 1e-6), with its FP64 figures reported.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from bp_gpu_util import BELIEF_TOL, MAP_MARGIN, STORAGE_LIMITED, STORAGE_LIMITED_SEEN, STORAGE_TOL, say
from synth_mrf import CONFIGS, make_batch_configs, make_batch_instance, make_config

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = ["stereo480x640_sum_sync", "stereo480x640_sum_checkerboard", "stereo480x640_max_sync",
         "stereo480x640_max_checkerboard", "stereo288x384_max_sync", "stereo288x384_max_checkerboard",
         "batch32_5_sum_sync", "batch32_3_sum_sync"]


def load(name):
    z = np.load(os.path.join(GOLDEN, f"e2e_{name}.npz"))
    return {k: z[k] for k in z.files if k != "meta"}, json.loads(str(z["meta"]))


def gpu_solve(meta, arith="f64", tuning=None):
    import torch
    src, mode, sched, n = meta["source"], meta["mode"], meta["schedule"], meta["n"]
    if src.startswith("batch:"):
        from paper_1010_0012_amd.batch import Batch
        j = int(src.split(":")[1])
        insts = make_batch_configs()
        gs = [torch.from_numpy(make_batch_instance(i)[0]).cuda() for i in insts]
        batch = Batch([(g, i.T, i.alpha) for g, i in zip(gs, insts)])
        batch.iterate(mode, n)
        b = batch.beliefs()[j].cpu().numpy()
        lab = batch.map_labels()[j].cpu().numpy()
        g32 = gs[j].cpu().numpy()
        torch.cuda.synchronize()
        batch.close()
        return g32, b, lab
    from paper_1010_0012_amd.grid import Grid
    cfg = CONFIGS[src]
    g32, _ = make_config(cfg)
    grid = Grid(cfg.H, cfg.W)
    grid.set_potential(cfg.M, cfg.T, cfg.alpha)
    grid.set_arithmetic(arith)
    grid.set_unary(torch.from_numpy(g32).cuda())
    if tuning:
        grid.set_launch_tuning(*tuning)
    grid.iterate(mode, n, sched)
    b = torch.empty((cfg.H, cfg.W, cfg.M), dtype=torch.float32, device="cuda")
    lab = torch.empty((cfg.H, cfg.W), dtype=torch.int32, device="cuda")
    grid.readout(b, lab)
    out = g32, b.cpu().numpy(), lab.cpu().numpy()
    torch.cuda.synchronize()
    grid.close()
    return out


def label_mismatches(lab, ref_labels, low_idx, low_margin):
    """Pixels whose label differs from the reference where the reference's
    margin exceeds 1e-6 (pixels outside low_idx have margins above 1e-4)."""
    diff = np.nonzero(lab.reshape(-1) != ref_labels.reshape(-1).astype(lab.dtype))[0]
    margin = dict(zip(low_idx.tolist(), low_margin.tolist()))
    return [(int(i), margin.get(int(i), np.inf)) for i in diff if margin.get(int(i), np.inf) > MAP_MARGIN]


@pytest.mark.parametrize("name", CASES)
def test_end_to_end(name):
    ref, meta = load(name)
    H, W, M = meta["H"], meta["W"], meta["M"]
    say(f"end-to-end {name}: {H}x{W} M={M} T={meta['T']} {meta['mode']} {meta['schedule']} x{meta['n']}")
    g32, b, lab = gpu_solve(meta)
    assert hashlib.sha256(np.ascontiguousarray(g32).tobytes()).hexdigest() == meta["unary_sha256"]
    np.testing.assert_array_equal(lab, np.argmax(b, axis=-1))
    bs = b.reshape(H * W, M)[ref["sample_idx"]]
    err = float(np.max(np.abs(bs - ref["sample_b"])))
    bad = label_mismatches(lab, ref["labels"], ref["low_idx"], ref["low_margin"])
    line = (f"{name}: FP64 max|db| on {len(ref['sample_idx'])} sampled pixels = {err:.2e}, MAP mismatches "
            f"(margin > 1e-6) = {len(bad)} of {H * W}; min FP64 margin {meta['min_margin']:.1e}")
    if "store_max_db" in meta:
        line += f"; float32-storage model alone: max|db| {meta['store_max_db']:.2e}, MAP flips {meta['store_map_mismatch']}"
    if "store_sample_b" in ref:
        err32 = float(np.max(np.abs(bs - ref["store_sample_b"])))
        bad32 = label_mismatches(lab, ref["store_labels"], ref["store_low_idx"], ref["store_low_margin"])
        line += f"; GPU vs the storage model: max|db| {err32:.2e}, MAP mismatches {len(bad32)}"
    say(line)
    limited = "store_max_db" in meta and (meta["store_max_db"] > BELIEF_TOL or meta["store_map_mismatch"] > 0)
    if name not in STORAGE_LIMITED:
        assert not limited or (err <= BELIEF_TOL and not bad), (
            f"{line}: the float32-storage model misses the FP64 bar on this case; name it in STORAGE_LIMITED")
        assert err <= BELIEF_TOL, line
        assert not bad, f"{line}; first mismatches (pixel, margin): {bad[:5]}"
        return
    assert limited, f"{name} is named storage-limited, but the float32-storage model meets the FP64 bar"
    say(f"{name} [storage-limited: {STORAGE_LIMITED[name]}]: FP64 bar NOT met by float32 storage; "
        f"vs the storage model max|db| = {err32:.2e}, MAP mismatches = {len(bad32)}")
    STORAGE_LIMITED_SEEN.append((name, err, len(bad), meta["store_max_db"]))
    assert err32 <= STORAGE_TOL, (name, err32)
    assert not bad32, (name, bad32[:5])


@pytest.mark.parametrize("name,layout", [("stereo480x640_sum_sync", "wide"), ("stereo480x640_sum_sync", "tile"),
                                         ("stereo480x640_sum_sync", "walk"),
                                         ("stereo480x640_sum_checkerboard", "wide")])
def test_end_to_end_f32_arithmetic(name, layout):
    """The 480x640 sum-product solves with float32 arithmetic against the
    FP64 oracle's solve: the bar itself (beliefs within 1e-5, MAP equal where
    the FP64 margin exceeds 1e-6), in the launch mappings the autotuner picks
    between (the tile launch is the one the benchmark's autotuning keeps)."""
    ref, meta = load(name)
    H, W, M = meta["H"], meta["W"], meta["M"]
    say(f"end-to-end {name}, float32 arithmetic, {layout}")
    g32, b, lab = gpu_solve(meta, arith="f32", tuning=(layout, -1))
    np.testing.assert_array_equal(lab, np.argmax(b, axis=-1))
    err = float(np.max(np.abs(b.reshape(H * W, M)[ref["sample_idx"]] - ref["sample_b"])))
    bad = label_mismatches(lab, ref["labels"], ref["low_idx"], ref["low_margin"])
    say(f"{name} [float32 arithmetic]: FP64 max|db| = {err:.2e}, MAP mismatches (margin > 1e-6) = {len(bad)}")
    assert err <= BELIEF_TOL
    assert not bad, bad[:5]
