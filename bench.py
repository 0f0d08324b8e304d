"""Throughput of the exact O(mM) BP message update on one MI355X.

One step = the whole single-grid hot path on the 480x640 synthetic stereo MRF
(M=64, T=4, alpha=0.5): set the potential, reset messages to 1/M, 100
synchronous sum-product iterations of the sparse update (Eq. 7), beliefs
(Eq. 3) and MAP labels.  Inputs are resident in HBM before timing starts.

value = directed-edge x label message updates per second over the timed
steps.  Beside it: max-product and checkerboard legs, the dense O(M^2)
comparison kernel, the dominant kernel's roofline (algorithmic bytes per
launch / HIP-event-timed average launch duration, against 8 TB/s), and the
FP64 oracle timed on a bounded sample on the host CPU.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-legs]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge·label msg updates/s, sparse O(mM) vs dense O(M²), % HBM peak; fwd+bwd it/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Legs beside the headline: other schedules and modes of the sparse update,
# the dense O(M^2) update, sweeps, coarse-to-fine, general potentials,
# factor graphs, the fbar = 0 experiment, forward + backward, batches.
LEGS = ("sparse", "dense", "sweep", "multiscale", "general", "factor", "fbar0", "grad", "batch", "walk")


def alg_bytes_per_sync_iter(cfg):
    """Each live message entry read once and written once, unary read once:
    4 * M * (2E + N) bytes per synchronous iteration."""
    return 4 * cfg.M * (2 * cfg.n_directed_edges + cfg.n_pixels)


KERNEL_SOURCES = ["paper_1010_0012_amd/csrc/bp_device.hpp", "paper_1010_0012_amd/csrc/bp_kernels.hpp",
                  "paper_1010_0012_amd/csrc/bp_sparse_dispatch.hpp", "paper_1010_0012_amd/csrc/bp_walk.hpp",
                  "paper_1010_0012_amd/csrc/bp_tile.hpp",
                  "paper_1010_0012_amd/csrc/bp_launch_sparse_sum.hip",
                  "paper_1010_0012_amd/csrc/bp_launch_sparse_sumf.hip",
                  "paper_1010_0012_amd/csrc/bp_launch_misc.hip"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "sparse_pair_tile_f32_stereo480x640.json")


def sparse_kernel_name(M, T, mode, pair=False, n_pixels=0, layout="wide"):
    """Template instance of the sparse update that runs (M, T): lanes per pixel
    G is the smallest power of two >= ceil(M/4) in [4, 64]; the window width is
    the smallest compiled half-width >= T; pair: the two-iteration launch,
    whose row-block form runs when M = 4G and the messages of one direction
    fit 32-bit byte offsets, unless the launch mapping is one group per
    pixel slot (mode 2: sum-product in float32 arithmetic, row blocks only);
    the column walk (synchronous, M = 32 or 64, planes below 2^31 bytes)
    or the tile launch (synchronous, M = 32 or 64) where the mapping is
    one of those."""
    G = 4
    while G * 4 < M and G < 64:
        G *= 2
    tws = (0, 1, 2, 3, 4, 6, 8, 12) + (() if G == 4 else (16,))
    tw = next((t for t in tws if t >= T), None)
    if tw is None:
        return f"sparse_update_wide_kernel<{G}, {mode}>"
    if pair and layout == "walk" and M == 4 * G and G in (8, 16) and n_pixels * M * 4 <= 2 ** 31:
        return f"sparse_walk2_kernel<{G}, {tw}, {mode}, 2>"
    if pair and layout == "tile" and M == 4 * G and G in (8, 16) and n_pixels * M * 4 < 2 ** 32:
        return f"sparse_tile2_kernel<{G}, {tw}, {mode}>"
    row_blocks = mode == 2 or layout != "slots"
    if pair and row_blocks and M == 4 * G and n_pixels * M * 4 < 2 ** 32:
        return f"sparse_update2_rows_kernel<{G}, {tw}, {mode}>"
    if pair:
        return f"sparse_update2_kernel<{G}, {tw}, {mode}, {'true' if M == 4 * G else 'false'}>"
    return f"sparse_update_kernel<{G}, {tw}, {mode}>"


def measured_traffic(kernel):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (each scaled by the same counter on a plain
    256 MiB copy), or None when the kernel sources changed since it was taken
    or the summary is of another kernel (another launch mapping)."""
    import hashlib
    try:
        rec = json.load(open(PMC_SUMMARY))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    same = rec.get("source_sha256") == h.hexdigest() and kernel in rec.get("kernel", "")
    return rec["traffic_bytes"] if same else None


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_accuracy(case, b, lab):
    """Error of a whole solve against the FP64 oracle's solve of the same
    workload, stored by tests/golden/make_e2e_ref.py (run on the CPU, oracle
    only): max |b - b_FP64| over the 4096 sampled pixels, MAP mismatches where
    the FP64 top-two margin exceeds 1e-6 (every pixel), and, where the file
    has it, the same for the oracle's float32-storage model alone."""
    import numpy as np
    try:
        z = np.load(os.path.join(GOLDEN, f"e2e_{case}.npz"))
    except OSError:
        return {}
    meta = json.loads(str(z["meta"]))
    H, W, M = meta["H"], meta["W"], meta["M"]
    bs = np.asarray(b).reshape(H * W, M)[z["sample_idx"]]
    lab = np.asarray(lab).reshape(-1)
    margin = dict(zip(z["low_idx"].tolist(), z["low_margin"].tolist()))
    diff = np.nonzero(lab != z["labels"].reshape(-1).astype(lab.dtype))[0]
    bad = sum(1 for i in diff if margin.get(int(i), math.inf) > 1e-6)
    out = {"case": case, "max_abs_db_vs_fp64": float(np.max(np.abs(bs - z["sample_b"]))),
           "map_mismatches_vs_fp64": int(bad), "pixels": H * W, "sampled_pixels": int(len(z["sample_idx"]))}
    if "store_max_db" in meta:
        out["f32_storage_model_max_abs_db_vs_fp64"] = meta["store_max_db"]
        out["max_abs_db_vs_f32_storage_model"] = float(np.max(np.abs(bs - z["store_sample_b"])))
    return out


def time_launches(grid, mode, n, schedule, dense, reps, iters_per_launch=1):
    """Average duration of one update launch (covering iters_per_launch
    iterations), from HIP events on the stream the library launches on
    (torch's current stream)."""
    import torch
    s = torch.cuda.current_stream()
    grid.reset()
    grid.iterate(mode, 2, schedule, dense=dense)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(reps):
        grid.reset()
        e0.record(s)
        grid.iterate(mode, n, schedule, dense=dense)
        e1.record(s)
        e1.synchronize()
        total += e0.elapsed_time(e1)
    return total * iters_per_launch / (reps * n)  # ms per launch


def run_meta(g32):
    """What the record was measured on: the input digest, the host CPU and
    its cores, the ROCm, HIP and torch versions."""
    import hashlib
    import platform

    import torch
    cpu = platform.processor()
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    rocm = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            rocm = fh.read().strip()
    except OSError:
        pass
    return {"input_sha256": hashlib.sha256(g32.tobytes()).hexdigest(), "host_cpu": cpu,
            "host_cores": os.cpu_count(), "rocm": rocm, "hip": torch.version.hip, "torch": torch.__version__,
            "device": torch.cuda.get_device_name(0)}


def cpu_baseline(cfg, g32, n_iters=5):
    """The FP64 oracle's sparse (Eq. 7) synchronous iterations on the full
    grid, one BLAS thread, timed on this host: a bounded sample of the
    workload (n_iters of its iterations, about 15 s)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import grid_bp as gb
    pot = gb.truncated_linear(cfg.M, cfg.T, cfg.alpha)
    g = g32.astype(np.float64)
    state = gb.init_messages(cfg.H, cfg.W, cfg.M)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(n_iters):
            state = gb.sync_step(g, state, pot, gb.SUM, gb.SPARSE)
        dt = time.perf_counter() - t0
    updates = cfg.n_directed_edges * cfg.M * n_iters
    return {"value": updates / dt, "unit": "edge·label updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_iters} synchronous sum-product iterations of the full {cfg.H}x{cfg.W} grid, "
                      f"M={cfg.M}, sparse Eq. 7 form, FP64 NumPy, 1 thread ({dt:.1f} s)"}


def grad_leg(reps=3):
    """Forward (with checkpoints) + backward of unrolled sum-product BP on the
    256x256, M=32, T=3, 30-iteration differentiation workload."""
    import torch

    from paper_1010_0012_amd import _lib as L
    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import CONFIGS, make_config
    cfg = CONFIGS["stereo256grad"]
    g32, y = make_config(cfg)
    grid = Grid(cfg.H, cfg.W)
    grid.set_potential(cfg.M, cfg.T, cfg.alpha)
    g = torch.from_numpy(g32).cuda()
    grid.set_unary(g)
    nbytes = L.bp_grad_workspace_bytes(grid.handle, cfg.iters, cfg.ckpt_every)
    gws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    yt = torch.from_numpy(y).cuda().long()
    b = torch.empty((cfg.H, cfg.W, cfg.M), dtype=torch.float32, device="cuda")
    dtheta = torch.empty_like(b)
    dalpha = torch.zeros(1, device="cuda")
    N = cfg.n_pixels

    def fwd_bwd():
        L.bp_forward_ckpt(grid.handle, cfg.iters, cfg.ckpt_every, gws, nbytes)
        grid.beliefs(b)
        by = torch.gather(b, -1, yt[..., None])
        dL_db = torch.zeros_like(b).scatter_(-1, yt[..., None], -1.0 / (N * by))
        L.bp_backward(grid.handle, dL_db, dtheta, dalpha)

    fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fwd_bwd()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    grid.close()
    log(f"bench: fwd+bwd {cfg.name}: {dt * 1e3:.2f} ms per {cfg.iters}-iteration forward+backward")
    out = {"fwd_bwd_workload": f"{cfg.name}: {cfg.H}x{cfg.W}, M={cfg.M}, T={cfg.T}, "
                               f"{cfg.iters} iterations, checkpoints every {cfg.ckpt_every}",
           "fwd_bwd_ms": dt * 1e3, "fwd_bwd_it_per_s": cfg.iters / dt,
           "fwd_bwd_solves_per_s": 1.0 / dt}
    # accuracy against the FP64 reference gradient (tests/golden, oracle only)
    import numpy as np
    try:
        z = np.load(os.path.join(GOLDEN, "grad_stereo256grad.npz"))
        meta = json.loads(str(z["meta"]))
        th = dtheta.cpu().numpy().reshape(-1, cfg.M)[z["sample_idx"]]
        out["fwd_bwd_accuracy"] = {
            "dtheta_max_abs_err_over_max_abs": float(np.max(np.abs(th - z["sample_dtheta"])) / meta["max_abs_dtheta"]),
            "dalpha_rel_err": abs(float(dalpha.cpu()[0]) - meta["dalpha"]) / abs(meta["dalpha"]),
            "sampled_pixels": int(len(z["sample_idx"])), "reference": "FP64 hand adjoint (oracle), 4096 sampled pixels"}
        log(f"bench: fwd+bwd accuracy {out['fwd_bwd_accuracy']}")
    except OSError:
        pass
    return out


def sweep_leg(grid, cfg, reps=2, arith="f32"):
    """Directional sweeps (Sec. 6): one sweep = passes left, right, up and down
    = every directed message once, sequential along each row or column.
    Time per sweep on the benchmark grid and at the paper's 144 x 192 shape
    (sparse vs dense there, beside the paper's CPU ratio of about 3.1), in
    double arithmetic, and the sparse sum-product sweep in float32 as well
    (_f32 keys).  The benchmark grid gets `arith` back afterwards."""
    import torch

    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import CONFIGS, make_config
    out = {}
    for name, c, gr in (("480x640", cfg, grid), ("144x192", CONFIGS["stereo144x192"], None)):
        own = gr is None
        if own:
            g32, _ = make_config(c)
            gr = Grid(c.H, c.W)
            gr.set_potential(c.M, c.T, c.alpha)
            gr.set_unary(torch.from_numpy(g32).cuda())
        updates = c.n_directed_edges * c.M
        for mode, dense, ar in (("sum", False, "f64"), ("max", False, "f64"), ("sum", True, "f64"),
                                ("sum", False, "f32")):
            gr.set_arithmetic(ar)
            ms = time_launches(gr, mode, 2, "sweep", dense, reps)  # ms per sweep
            key = f"sweep_{name}_{'dense' if dense else 'sparse'}_{mode}" + ("_f32" if ar == "f32" else "")
            out[key + "_us"] = ms * 1e3
            out[key + "_updates_per_s"] = updates / (ms * 1e-3)
            log(f"bench: {key}: {ms * 1e3:.1f} us/sweep, {updates / (ms * 1e-3):.3e} updates/s")
        out[f"sweep_{name}_dense_over_sparse_sum"] = out[f"sweep_{name}_dense_sum_us"] / out[f"sweep_{name}_sparse_sum_us"]
        if own:
            gr.close()
        else:
            gr.set_arithmetic(arith)
    return out


def fbar_zero_leg():
    """Sec. 6's f-bar = 0 experiment on the synthetic 144 x 192 stereo pair:
    ten sum-product sweeps with f-bar = exp(-alpha T) and with f-bar = 0;
    the fraction of disparity labels that change, and each map's error rate
    against the synthetic ground truth (|label - disparity| > 1)."""
    import numpy as np
    import torch

    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import CONFIGS, make_config
    c = CONFIGS["stereo144x192"]
    g32, D = make_config(c)
    labels = {}
    for name, fbar in (("tied", None), ("zero", 0.0)):
        gr = Grid(c.H, c.W)
        gr.set_potential(c.M, c.T, c.alpha, fbar)
        gr.set_unary(torch.from_numpy(g32).cuda())
        gr.iterate("sum", c.iters, "sweep")
        labels[name] = gr.map_labels().cpu().numpy()
        gr.close()
    changed = float(np.mean(labels["tied"] != labels["zero"]))
    bad = {k: float(np.mean(np.abs(v.astype(np.int64) - D) > 1)) for k, v in labels.items()}
    log(f"bench: fbar=0 experiment (144x192, {c.iters} sweeps): {100 * changed:.2f}% of labels change; "
        f"bad pixels {100 * bad['tied']:.2f}% (fbar=exp(-aT)) vs {100 * bad['zero']:.2f}% (fbar=0)")
    return {"fbar0_labels_changed": changed, "fbar0_bad_pixels_tied": bad["tied"],
            "fbar0_bad_pixels_zero": bad["zero"]}


def multiscale_leg(grid, cfg, reps=3):
    """Coarse-to-fine BP with the O(mM) update (Sec. 2, Sec. 6) on the
    benchmark grid: three coarser levels with 10 iterations each and n0 at
    the finest, against plain BP with the same finest-level work.  Quality
    is the largest belief difference from the 100-iteration plain solve (the
    workload's own result) and the share of labels that differ from it."""
    import numpy as np
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    grid.reset()
    grid.iterate("sum", cfg.iters)
    ref_b = grid.beliefs().cpu().numpy()
    ref_l = grid.map_labels().cpu().numpy()
    out = {}
    for n0 in (10, 25):
        for name, run in (("multiscale", lambda: grid.iterate_multiscale("sum", [n0, 10, 10, 10])),
                          ("plain", lambda: (grid.reset(), grid.iterate("sum", n0)))):
            run()
            torch.cuda.synchronize()
            ms_best = 1e30
            for _ in range(reps):
                e0.record(s)
                run()
                e1.record(s)
                e1.synchronize()
                ms_best = min(ms_best, e0.elapsed_time(e1))
            b = grid.beliefs().cpu().numpy()
            lab = grid.map_labels().cpu().numpy()
            db = float(np.max(np.abs(b - ref_b)))
            dl = float(np.mean(lab != ref_l))
            key = f"{name}_n0_{n0}"
            out[key + "_ms"] = ms_best
            out[key + "_max_db_vs_100"] = db
            out[key + "_labels_differ_vs_100"] = dl
            log(f"bench: {key}: {ms_best:.2f} ms, max|b - b100| = {db:.3e}, labels differing from the "
                f"100-iteration solve {100 * dl:.2f}%")
    return out


def general_leg(g, cfg, n_iters=20, reps=2):
    """General sparse compatibility (Sec. 4, Sec. 7) on the benchmark grid:
    the general kernel on (a) the truncated-linear potential given as a CSR
    table (against the window kernel on the same problem), (b) four random
    potential types on the edges, each with about 2T+1 compatible labels
    per label, and (c) max-product with fbar above f(T) (Eq. 10)."""
    import numpy as np
    import torch

    from paper_1010_0012_amd.grid import Grid
    H, W, M, T = cfg.H, cfg.W, cfg.M, cfg.T
    updates = cfg.n_directed_edges * M
    a32 = float(np.float32(cfg.alpha))
    fbar = float(np.float32(np.exp(-a32 * T)))

    def window_csr(fb):
        col_ptr, row_idx, val = [0], [], []
        for y in range(M):
            for x in range(max(0, y - T), min(M - 1, y + T) + 1):
                row_idx.append(x)
                val.append(np.float32(np.exp(-a32 * abs(x - y))))
            col_ptr.append(len(row_idx))
        return np.array(col_ptr), np.array(row_idx), np.array(val, dtype=np.float32), fb

    rng = np.random.default_rng(17)

    def random_csr():
        col_ptr, row_idx, val = [0], [], []
        for y in range(M):
            xs = np.sort(rng.choice(M, size=2 * T + 1, replace=False))
            row_idx += xs.tolist()
            val += rng.uniform(0.3, 1.0, len(xs)).astype(np.float32).tolist()
            col_ptr.append(len(row_idx))
        return np.array(col_ptr), np.array(row_idx), np.array(val, dtype=np.float32), 0.1

    th = torch.from_numpy(rng.integers(0, 4, (H, W - 1)).astype(np.uint8)).cuda()
    tv = torch.from_numpy(rng.integers(0, 4, (H - 1, W)).astype(np.uint8)).cuda()
    cases = [("window_as_csr_sum", "sum", None, [window_csr(fbar)], None),
             ("window_as_csr_max", "max", None, [window_csr(fbar)], None),
             ("four_types_sum", "sum", None, [random_csr() for _ in range(4)], (th, tv)),
             ("four_types_max", "max", None, [random_csr() for _ in range(4)], (th, tv)),
             ("eq10_window_max", "max", 1.5 * fbar, None, None)]
    out = {}
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, mode, fb, types, maps in cases:
        grid = Grid(H, W)
        grid.set_potential(M, T, cfg.alpha, fb)
        if types is not None:
            grid.set_sparse_potentials(types, *(maps or (None, None)))
        grid.set_unary(g)
        grid.iterate(mode, 2)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            e0.record(s)
            grid.iterate(mode, n_iters)
            e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / n_iters)
        grid.close()
        out[f"general_{name}_us_per_iter"] = best * 1e3
        out[f"general_{name}_updates_per_s"] = updates / (best * 1e-3)
        log(f"bench: general {name}: {best * 1e3:.1f} us per iteration, {updates / (best * 1e-3):.3e} updates/s")
    return out


def factor_leg(reps=3, n_iters=10):
    """Higher-order factors (Sec. 7): a 256 x 256 grid of variables, M = 32,
    triple factors along every row and column with a second-order smoothness
    compatibility (1094 of the 32768 triples), sum-product; the O(C + M)
    update against the plain O(M^3) one (every triple listed) on the same
    graph.  Updates counted as factor->variable label entries."""
    import torch

    from paper_1010_0012_amd.factor import FactorGraph
    from synth_mrf import make_factor_grid
    spec = make_factor_grid(256, 256, 32, seed=9)
    G = FactorGraph(spec.n_vars, spec.M, spec.factor_vars, spec.factor_type, spec.types, dense_tables=True)
    G.set_unary(torch.from_numpy(spec.unary).cuda())
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    updates = len(spec.factor_type) * 3 * spec.M
    out = {"factor_workload": "256x256 variables, M=32, 130,048 triple factors, C=1094 of 32768, sum-product"}
    for dense in (False, True):
        G.reset()
        G.iterate("sum", 2, dense=dense)
        best = 1e30
        for _ in range(reps):
            e0.record(s)
            G.iterate("sum", n_iters, dense=dense)
            e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / n_iters)
        key = "factor_dense" if dense else "factor_sparse"
        out[key + "_ms_per_iter"] = best
        out[key + "_updates_per_s"] = updates / (best * 1e-3)
        log(f"bench: {key}: {best * 1e3:.1f} us per iteration, {updates / (best * 1e-3):.3e} updates/s")
    out["factor_dense_over_sparse"] = out["factor_dense_ms_per_iter"] / out["factor_sparse_ms_per_iter"]
    G.close()
    return out


def walk_leg(reps=5, n_iters=20):
    """The two-iteration launch on a 480 x 640 grid with M = 32 (T = 3,
    alpha = 0.5, float32 arithmetic, seeded uniform unary): wide column
    strips, the column walk (each grid row staged once in LDS) and the tile
    launch (4 x 8 pixel tiles and their halo staged in LDS), per launch, and
    what the autotuner picks.  Algorithmic bytes 4 M (2E + N)."""
    import torch

    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import random_unary
    H, W, M, T = 480, 640, 32, 3
    grid = Grid(H, W)
    grid.set_potential(M, T, 0.5)
    grid.set_arithmetic("f32")
    grid.set_unary(torch.from_numpy(random_unary(H, W, M, 3)).cuda())
    alg = 4 * M * (2 * (2 * H * W - H - W) * 2 + H * W)
    out = {"walk_workload": f"{H}x{W}, M={M}, T={T}, sum-product sync, float32 arithmetic, pair launches"}
    for layout in ("wide", "walk", "tile"):
        grid.set_launch_tuning(layout, -1)
        best = min(time_launches(grid, "sum", n_iters, "sync", False, 1, iters_per_launch=2) for _ in range(reps))
        out[f"walk_leg_{layout}_pair_launch_us"] = best * 1e3
        out[f"walk_leg_{layout}_GBs"] = alg / (best * 1e-3) / 1e9
        log(f"bench: {H}x{W}x{M} pair launch, {layout}: {best * 1e3:.1f} us ({alg / (best * 1e-3) / 1e9:.0f} GB/s)")
    grid.set_launch_tuning("wide", -1)
    grid.autotune("sum", "sync", 4)
    out["walk_leg_autotuned"] = list(grid.get_launch_tuning())
    out["walk_leg_wide_over_walk"] = out["walk_leg_wide_pair_launch_us"] / out["walk_leg_walk_pair_launch_us"]
    out["walk_leg_wide_over_tile"] = out["walk_leg_wide_pair_launch_us"] / out["walk_leg_tile_pair_launch_us"]
    grid.close()
    return out


def batch_leg(arith="f64", n_iters=30, reps=3):
    """The 32-instance batch (H, W in [64, 512], M in {16, 32, 64, 128}, T in
    [1, 8]) in the given arithmetic: autotuned plan, n_iters sum-product
    iterations per graph replay; each label class (the instances of one M)
    as a batch of its own; and the same instances run one grid at a time.
    Double by default: float32 arithmetic ends 1.3e-5 from the FP64 solve on
    the smallest instance (78 x 115, M = 32), beyond the 1e-5 bar."""
    import torch

    from paper_1010_0012_amd.batch import Batch
    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import make_batch_configs, make_batch_instance
    insts = make_batch_configs()
    gs = [torch.from_numpy(make_batch_instance(i)[0]).cuda() for i in insts]
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def work(js):
        updates = sum(2 * (insts[j].H * (insts[j].W - 1) + insts[j].W * (insts[j].H - 1)) * insts[j].M
                      for j in js) * n_iters
        # one synchronous iteration's bytes (each message read and written once,
        # the unary read once); a two-iteration launch moves one iteration's bytes
        iter_bytes = sum(4 * insts[j].M * (2 * 2 * (insts[j].H * (insts[j].W - 1) + insts[j].W * (insts[j].H - 1))
                                           + insts[j].H * insts[j].W) for j in js) * n_iters
        return updates, iter_bytes

    def run_batch(js):
        batch = Batch([(gs[j], insts[j].T, insts[j].alpha) for j in js])
        batch.set_arithmetic(arith)
        best_us = batch.autotune("sum", 2)
        batch.reset()
        batch.iterate("sum", n_iters)          # captures the graph
        torch.cuda.synchronize()
        ms = 1e30
        for _ in range(reps):
            batch.reset()
            e0.record(s)
            batch.iterate("sum", n_iters)
            e1.record(s)
            e1.synchronize()
            ms = min(ms, e0.elapsed_time(e1))
        return batch, ms, best_us

    every = list(range(len(insts)))
    batch, ms, best_us = run_batch(every)
    plan = batch.get_plan()
    streams = batch.get_streams()
    updates, iter_bytes = work(every)
    acc = {}
    j = min(every, key=lambda i: insts[i].H * insts[i].W * insts[i].M)
    b_j, l_j = batch.beliefs()[j].cpu().numpy(), batch.map_labels()[j].cpu().numpy()
    acc[f"batch32_{j}_sum_sync"] = golden_accuracy(f"batch32_{j}_sum_sync", b_j, l_j)
    j = max((i for i in every if insts[i].M == 128), key=lambda i: insts[i].H * insts[i].W)
    b_j, l_j = batch.beliefs()[j].cpu().numpy(), batch.map_labels()[j].cpu().numpy()
    acc[f"batch32_{j}_sum_sync"] = golden_accuracy(f"batch32_{j}_sum_sync", b_j, l_j)
    log(f"bench: batch accuracy {acc}")
    batch.close()
    # each label class as a batch of its own
    classes = {}
    for M in sorted({i.M for i in insts}):
        js = [j for j in every if insts[j].M == M]
        cb, cms, _ = run_batch(js)
        cb.close()
        cu, cbytes = work(js)
        classes[f"M{M}"] = {"instances": len(js), "ms": cms, "updates_per_s": cu / (cms * 1e-3),
                            "iteration_equiv_GBs": cbytes / (cms * 1e-3) / 1e9,
                            "launch_GBs": cbytes / 2 / (cms * 1e-3) / 1e9}
        log(f"bench: batch class M={M}: {len(js)} instances, {cms:.2f} ms, "
            f"{cbytes / 2 / (cms * 1e-3) / 1e9:.0f} GB/s on the pair launches' own bytes")
    # one grid at a time (the best of `reps` solves of each)
    t_single = 0.0
    for g, i in zip(gs, insts):
        grid = Grid(i.H, i.W)
        grid.set_potential(i.M, i.T, i.alpha)
        grid.set_arithmetic(arith)
        grid.set_unary(g)
        grid.iterate("sum", 2)
        best = 1e30
        for _ in range(reps):
            grid.reset()
            e0.record(s)
            grid.iterate("sum", n_iters)
            e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        t_single += best
        grid.close()
    log(f"bench: batch32 x{n_iters} ({arith}): {ms:.2f} ms ({updates / (ms * 1e-3):.4e} updates/s, "
        f"{iter_bytes / 2 / (ms * 1e-3) / 1e9:.0f} GB/s on the pair launches' own bytes), plan {plan}, "
        f"{streams} streams; one grid at a time {t_single:.2f} ms ({t_single / ms:.2f}x)")
    return {"batch_workload": f"32 grids, H,W in [64,512], M in {{16,32,64,128}}, T in [1,8], "
                              f"{n_iters} sum-product iterations, one graph replay, {arith} arithmetic",
            "batch_ms": ms, "batch_updates_per_s": updates / (ms * 1e-3),
            "batch_alg_GBs": iter_bytes / (ms * 1e-3) / 1e9,
            "batch_launch_GBs": iter_bytes / 2 / (ms * 1e-3) / 1e9,
            "batch_plan": {"passes": plan[0], "grid_blocks": plan[1], "streams": streams, "autotune_best_us": best_us},
            "batch_one_grid_at_a_time_ms": t_single, "batch_over_one_at_a_time": t_single / ms,
            "batch_classes": classes, "batch_accuracy": acc}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip every leg beside the headline")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help=f"comma-separated legs to run beside the headline, of {','.join(LEGS)}")
    ap.add_argument("--tuning", default=None,
                    help="LAYOUT:CAP launch mapping of the headline (e.g. wide:-1) instead of autotuning it")
    ap.add_argument("--arith", choices=("f32", "f64"), default="f32",
                    help="arithmetic of the headline sum-product update (bp_set_arithmetic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1010_0012_amd.grid import Grid
    from synth_mrf import CONFIGS, make_config

    cfg = CONFIGS["stereo480x640"]
    g32, _ = make_config(cfg)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    g = torch.from_numpy(g32).to(dev)
    grid = Grid(cfg.H, cfg.W)
    grid.set_potential(cfg.M, cfg.T, cfg.alpha)
    grid.set_arithmetic(args.arith)
    grid.set_unary(g)
    # the two-iteration launch's mapping: timed on this grid (bp_autotune), or given
    if args.tuning:
        layout, cap = args.tuning.split(":")
        grid.set_launch_tuning(layout, int(cap))
        tune_us = None
    else:
        tune_us = grid.autotune("sum", "sync", 10)
    tuning = grid.get_launch_tuning()
    launch_tuning = {args.arith: {"layout": tuning[0], "cap": tuning[1], "autotune_us_per_iteration": tune_us}}
    log(f"bench: launch mapping {tuning}" + (f" (autotuned: {tune_us:.1f} us per iteration in the trial)"
                                               if tune_us is not None else " (given)"))
    beliefs = torch.empty((cfg.H, cfg.W, cfg.M), dtype=torch.float32, device=dev)
    labels = torch.empty((cfg.H, cfg.W), dtype=torch.int32, device=dev)
    updates_per_iter = cfg.n_directed_edges * cfg.M

    def step(mode="sum", schedule="sync", dense=False):
        grid.set_potential(cfg.M, cfg.T, cfg.alpha)
        grid.reset()
        n = cfg.iters if schedule == "sync" else 2 * cfg.iters
        grid.iterate(mode, n, schedule, dense=dense)
        grid.readout(beliefs, labels)

    log(f"bench: {cfg.name} {cfg.H}x{cfg.W} M={cfg.M} T={cfg.T} iters={cfg.iters}, {args.arith} arithmetic")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = updates_per_iter * cfg.iters * args.steps / dt
    log(f"bench: sum sync {ms_per_step:.3f} ms/step, {value:.4e} updates/s")
    accuracy = golden_accuracy(f"{cfg.name}_sum_sync", beliefs.cpu().numpy(), labels.cpu().numpy())
    log(f"bench: accuracy of the last step vs the FP64 oracle's solve: {accuracy}")

    # Dominant kernel: the sparse sum-product launch that runs two synchronous
    # iterations; per launch it reads the unary and the inbox once and writes
    # the outbox once, the same bytes as a one-iteration launch.
    reps = max(2, args.steps)
    ms_launch = time_launches(grid, "sum", cfg.iters, "sync", False, reps, iters_per_launch=2)
    bytes_launch = alg_bytes_per_sync_iter(cfg)
    achieved = bytes_launch / (ms_launch * 1e-3) / 1e9
    per_iter_equiv = bytes_launch / (ms_launch / 2 * 1e-3) / 1e9
    kernel = sparse_kernel_name(cfg.M, cfg.T, 2 if args.arith == "f32" else 0, pair=True, n_pixels=cfg.n_pixels,
                                layout=tuning[0])
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel),
                "kernel": kernel,
                "launch_mapping": {"layout": tuning[0], "cap": tuning[1]},
                "arithmetic": args.arith,
                "alg_bytes_per_launch": bytes_launch, "avg_launch_us": ms_launch * 1e3,
                "iterations_per_launch": 2,
                # one iteration's algorithmic bytes (the per-iteration model:
                # every message read and written once, the unary read once)
                # over the launch time per iteration; above 1 because the
                # first iteration's messages never reach HBM
                "frac_per_iteration_equiv": per_iter_equiv / HBM_PEAK_GBS}
    log(f"bench: sparse sum pair launch {ms_launch * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic "
        f"({100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s)")

    extra = {"sparse_sum_sync_pair_launch_us": ms_launch * 1e3, "accuracy": accuracy, "run": run_meta(g32)}
    # one iteration per launch, for comparison
    grid.set_sync_fusion(False)
    ms_single = time_launches(grid, "sum", cfg.iters, "sync", False, reps)
    grid.set_sync_fusion(True)
    extra["sparse_sum_sync_single_launch_us"] = ms_single * 1e3
    extra["sparse_sum_sync_single_launch_GBs"] = bytes_launch / (ms_single * 1e-3) / 1e9
    extra["sparse_sum_sync_single_launch_frac"] = bytes_launch / (ms_single * 1e-3) / 1e9 / HBM_PEAK_GBS
    extra["pair_over_single_per_iteration"] = ms_single / (ms_launch / 2)
    # one iteration's algorithmic bytes over the pair launch's time per
    # iteration: above the HBM peak means the pair beats the one-iteration
    # roofline (its first iteration's messages never reach HBM)
    extra["sparse_sum_sync_pair_per_iteration_equiv_GBs"] = bytes_launch / (ms_launch / 2 * 1e-3) / 1e9
    extra["sparse_sum_sync_pair_per_iteration_equiv_frac"] = bytes_launch / (ms_launch / 2 * 1e-3) / 1e9 / HBM_PEAK_GBS
    log(f"bench: sparse sum single launch {ms_single * 1e3:.1f} us "
        f"({bytes_launch / (ms_single * 1e-3) / 1e9:.0f} GB/s); pair launch per iteration {ms_launch * 500:.1f} us")
    # the other arithmetic beside it (double: every message its exact value rounded once)
    other = "f64" if args.arith == "f32" else "f32"
    grid.set_arithmetic(other)
    if not args.tuning:
        grid.set_launch_tuning("wide", -1)  # tuned from the default, not from the other arithmetic's choice
    o_us = grid.autotune("sum", "sync", 10) if not args.tuning else None
    o_tuning = grid.get_launch_tuning()
    launch_tuning[other] = {"layout": o_tuning[0], "cap": o_tuning[1], "autotune_us_per_iteration": o_us}
    extra["launch_tuning"] = launch_tuning
    ms_o = time_launches(grid, "sum", cfg.iters, "sync", False, reps, iters_per_launch=2)
    grid.readout(beliefs, labels)
    extra[f"sparse_sum_sync_{other}_pair_launch_us"] = ms_o * 1e3
    extra[f"sparse_sum_sync_{other}_pair_launch_frac"] = bytes_launch / (ms_o * 1e-3) / 1e9 / HBM_PEAK_GBS
    extra[f"sparse_sum_sync_{other}_accuracy"] = golden_accuracy(f"{cfg.name}_sum_sync", beliefs.cpu().numpy(),
                                                                labels.cpu().numpy())
    grid.set_sync_fusion(False)
    extra[f"sparse_sum_sync_{other}_single_launch_us"] = time_launches(grid, "sum", cfg.iters, "sync", False,
                                                                      reps) * 1e3
    grid.set_sync_fusion(True)
    grid.set_arithmetic(args.arith)
    grid.set_launch_tuning(*tuning)
    log(f"bench: {other} arithmetic: pair launch {ms_o * 1e3:.1f} us, single launch "
        f"{extra[f'sparse_sum_sync_{other}_single_launch_us']:.1f} us")
    legs = set() if args.no_legs else {x for x in args.legs.split(",") if x}
    unknown = legs - set(LEGS)
    if unknown:
        raise SystemExit(f"bench.py: unknown legs {sorted(unknown)}; known: {','.join(LEGS)}")
    schedule_legs = []
    if "sparse" in legs:
        schedule_legs += [("max", "sync", False), ("sum", "checkerboard", False), ("max", "checkerboard", False)]
    if "dense" in legs:
        schedule_legs += [("sum", "sync", True), ("max", "sync", True)]
    if schedule_legs:
        for mode, sched, dense in schedule_legs:
            # sparse launches run two iterations (sync) or two passes
            # (checkerboard) each; dense launches run one
            n = cfg.iters if sched == "sync" else 2 * cfg.iters
            per_launch = 1 if dense else 2
            key = f"{'dense' if dense else 'sparse'}_{mode}_{sched}"
            if not dense and args.tuning is None:
                # the sparse launches' mapping, tuned for this mode and schedule
                grid.autotune(mode, sched, 4)
                extra[key + "_launch_mapping"] = list(grid.get_launch_tuning())
            ms = time_launches(grid, mode, n, sched, dense, 2, iters_per_launch=per_launch)
            step = ms / per_launch                                   # one iteration or one pass
            per_iter = step * (1 if sched == "sync" else 2)          # every message updated once
            unit = "iteration" if sched == "sync" else "pass"
            # the state is that of a whole solve from the uniform start
            grid.readout(beliefs, labels)
            extra[key + "_accuracy"] = golden_accuracy(f"{cfg.name}_{mode}_{sched}", beliefs.cpu().numpy(),
                                                       labels.cpu().numpy())
            extra[key + "_updates_per_s"] = updates_per_iter / (per_iter * 1e-3)
            extra[key + "_launch_us"] = ms * 1e3
            extra[key + f"_us_per_{unit}"] = step * 1e3
            log(f"bench: {key}: {ms * 1e3:.1f} us per launch, {step * 1e3:.1f} us per {unit}, "
                f"{updates_per_iter / (per_iter * 1e-3):.4e} updates/s")
        grid.set_launch_tuning(*tuning)  # the headline's mapping for the legs that follow
    if {"sparse", "dense"} <= legs:
        # sparse O(mM) against dense O(M^2), like for like: one iteration per
        # launch on both sides, and each side's fastest form (the sparse pair
        # launch per iteration; the dense kernel has no pair form); both in
        # double arithmetic (the dense sum-product runs on the FP64 matrix
        # cores), with the dense kernels' own FP64 fraction
        grid.set_arithmetic("f64")
        grid.set_sync_fusion(False)
        extra["sparse_max_sync_single_launch_us"] = time_launches(grid, "max", cfg.iters, "sync", False, 2) * 1e3
        grid.set_sync_fusion(True)
        extra["sparse_sum_sync_f64_pair_per_iteration_us"] = (
            extra.get("sparse_sum_sync_f64_pair_launch_us", ms_launch * 1e3) / 2)
        grid.set_arithmetic(args.arith)
        flops = 2.0 * cfg.n_directed_edges * cfg.M * cfg.M          # Eq. 2 / Eq. 9 per iteration
        single = {"sum": extra.get("sparse_sum_sync_f64_single_launch_us", ms_single * 1e3),
                  "max": extra["sparse_max_sync_single_launch_us"]}
        best = {"sum": extra["sparse_sum_sync_f64_pair_per_iteration_us"],
                "max": extra["sparse_max_sync_us_per_iteration"]}
        for mode in ("sum", "max"):
            d_us = extra[f"dense_{mode}_sync_us_per_iteration"]
            extra[f"dense_{mode}_sync_fp64_TFs"] = flops / (d_us * 1e-6) / 1e12
            extra[f"dense_{mode}_sync_frac_fp64_peak"] = flops / (d_us * 1e-6) / 78.6e12
            extra[f"sparse_over_dense_{mode}_single_vs_single"] = d_us / single[mode]
            extra[f"sparse_over_dense_{mode}_best_vs_best"] = d_us / best[mode]
            log(f"bench: sparse over dense ({mode}): {d_us / single[mode]:.2f}x single vs single, "
                f"{d_us / best[mode]:.2f}x best vs best; dense at {flops / (d_us * 1e-6) / 1e12:.1f} TF/s "
                f"({100 * flops / (d_us * 1e-6) / 78.6e12:.0f}% of the FP64 peak)")
        extra["sparse_over_dense_target"] = cfg.M / (2 * cfg.T + 1) * 0.5
    for name, leg in (("sweep", lambda: sweep_leg(grid, cfg, arith=args.arith)), ("multiscale", lambda: multiscale_leg(grid, cfg)),
                      ("general", lambda: general_leg(g, cfg)), ("factor", factor_leg), ("fbar0", fbar_zero_leg),
                      ("grad", grad_leg), ("batch", batch_leg), ("walk", walk_leg)):
        if name in legs:
            extra.update(leg())

    # copy-kernel ceiling on this GPU (torch device-to-device copy)
    big = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(big)
    dst.copy_(big)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(big)
    e1.record()
    e1.synchronize()
    extra["copy_GBs"] = 2 * big.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del big, dst

    cpu = None
    if not args.no_cpu:
        log("bench: timing the FP64 oracle on the host (bounded sample)")
        cpu = cpu_baseline(cfg, g32)
        log(f"bench: cpu oracle {cpu['value']:.3e} updates/s")

    grid.close()
    out = {
        "metric": METRIC, "value": value, "unit": "edge·label updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.arith,
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.H}x{cfg.W} grid, M={cfg.M}, T={cfg.T}, "
                               f"alpha={cfg.alpha}, {cfg.iters} synchronous sum-product iterations "
                               f"(sparse O(mM) update, {args.arith} arithmetic, float32 messages) + beliefs + MAP",
                   "H": cfg.H, "W": cfg.W, "M": cfg.M, "T": cfg.T, "iters": cfg.iters,
                   "mode": "sum", "schedule": "sync", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
