"""Write the end-to-end reference files tests/golden/e2e_<case>.npz.

Each case is a whole solve of one synthetic workload, run by the FP64 oracle
alone (nothing here touches the HIP library): uniform start, n iterations
(synchronous) or passes (checkerboard), then Eq. 3 beliefs and the MAP labels
(Sec. 6 disparity map).  The GPU tests compare a full GPU solve of the same
workload, in the launch configuration the benchmark uses, with these files.

Per case the file holds
  labels       uint8 [H, W]   FP64 MAP labels, every pixel (lowest label on ties)
  low_idx      int32 [k]      flat indices of the pixels whose top-two belief
  low_margin   float64 [k]    margin is <= 1e-4, and those margins (every other
                              pixel's margin is larger)
  sample_idx   int32 [4096]   a fixed sample of pixels: the four corners, 128
                              on each border, the 512 lowest-margin pixels, the
                              512 pixels where float32 message storage moves the
                              beliefs most (when the storage run exists), the
                              rest uniform
  sample_b     float64 [4096, M]  FP64 beliefs at the sample
  store_labels, store_low_idx, store_low_margin, store_sample_b
                              the same for the float32-storage model's solve
                              (its sampled beliefs rounded to float32)
  min_margin, and (with the storage run) store_max_db / store_map_mismatch:
                              how far the oracle's float32-storage model (every
                              message computed in FP64 from stored float32
                              values and rounded once to float32) ends from FP64
                              over all pixels, the quantity that tells whether
                              float32 messages can meet the 1e-5 bar at all.

Sum-product cases run the dense Eq. 2 form (the method's definition, through
one matrix product per direction); max-product cases run the sparse Eq. 11
form, which equals Eq. 9 bit for bit when f >= fbar (the oracle's exactness
pins).  The potential is the one the C ABI documents holding (float32 alpha;
float32 table values for max-product).

Usage: python tests/golden/make_e2e_ref.py [--jobs 8] [--scratch DIR] [case ...]
       python tests/golden/make_e2e_ref.py --assemble [--scratch DIR]
       python tests/golden/make_e2e_ref.py --grad       (the gradient reference)
A case's runs take from seconds (288x384) to about 90 minutes (480x640
max-product checkerboard, 200 passes) on one core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

from oracle import grid_bp as gb  # noqa: E402
from synth_mrf import CONFIGS, make_batch_configs, make_batch_instance, make_config  # noqa: E402

N_SAMPLE = 4096
LOW_MARGIN = 1e-4


def library_potential(M, T, alpha, mode):
    """The tied potential as the C ABI holds it: alpha rounded to float32;
    sum-product f(d) = exp(-alpha |d|) and fbar = f(T) in double; max-product
    the float32 values of f(d) and fbar."""
    alpha = float(np.float32(alpha))
    pot = gb.truncated_linear(M, T, alpha)
    if mode == gb.MAX:
        f32 = float(np.float32(np.exp(-alpha * T)))
        F = np.where(pot.compat, pot.F.astype(np.float32).astype(np.float64), f32)
        pot = gb.Potential(F, pot.compat, f32)
    return pot


def case_list():
    """name -> (unary maker, M, T, alpha, mode, schedule, n, storage run wanted)."""
    out = {}
    c2 = CONFIGS["stereo480x640"]
    c1 = CONFIGS["stereo288x384"]
    for mode in (gb.SUM, gb.MAX):
        for sched in (gb.SYNC, gb.CHECKERBOARD):
            n = c2.iters if sched == gb.SYNC else 2 * c2.iters
            out[f"stereo480x640_{mode}_{sched}"] = ("stereo480x640", c2.M, c2.T, c2.alpha, mode, sched, n,
                                                    mode == gb.MAX)
    for sched in (gb.SYNC, gb.CHECKERBOARD):
        n = c1.iters if sched == gb.SYNC else 2 * c1.iters
        out[f"stereo288x384_max_{sched}"] = ("stereo288x384", c1.M, c1.T, c1.alpha, gb.MAX, sched, n, True)
    insts = make_batch_configs()
    j = max((i for i in range(len(insts)) if insts[i].M == 128), key=lambda i: insts[i].H * insts[i].W)
    it = insts[j]
    out[f"batch32_{j}_sum_sync"] = (f"batch:{j}", it.M, it.T, it.alpha, gb.SUM, gb.SYNC, 30, True)
    j = min(range(len(insts)), key=lambda i: insts[i].H * insts[i].W * insts[i].M)   # the smallest instance
    it = insts[j]
    out[f"batch32_{j}_sum_sync"] = (f"batch:{j}", it.M, it.T, it.alpha, gb.SUM, gb.SYNC, 30, True)
    return out


def write_grad_ref():
    """tests/golden/grad_stereo256grad.npz: the FP64 reference gradient of the
    256 x 256, M = 32, T = 3, 30-iteration differentiation workload (mean
    cross-entropy of the beliefs against the ground-truth disparity): the
    loss, dL/dalpha, max |dL/dtheta| and dL/dtheta at 4096 seeded pixels
    (the GPU's relative error is max |difference| / max |dL/dtheta|)."""
    from threadpoolctl import threadpool_limits

    from oracle import grad_ref
    cfg = CONFIGS["stereo256grad"]
    g32, y = make_config(cfg)
    t0 = time.time()
    with threadpool_limits(limits=1):
        L, dtheta, dalpha = grad_ref.grad(g32.astype(np.float64), y, cfg.M, cfg.T, float(np.float32(cfg.alpha)),
                                         cfg.iters)
    idx = np.sort(np.random.default_rng(2025).choice(cfg.H * cfg.W, N_SAMPLE, replace=False)).astype(np.int32)
    meta = {"case": "stereo256grad", "H": cfg.H, "W": cfg.W, "M": cfg.M, "T": cfg.T,
            "alpha_f32": float(np.float32(cfg.alpha)), "n": cfg.iters, "loss": float(L), "dalpha": float(dalpha),
            "max_abs_dtheta": float(np.max(np.abs(dtheta))),
            "unary_sha256": hashlib.sha256(np.ascontiguousarray(g32).tobytes()).hexdigest()}
    out = os.path.join(HERE, "grad_stereo256grad.npz")
    np.savez_compressed(out, sample_idx=idx, sample_dtheta=dtheta.reshape(-1, cfg.M)[idx], meta=json.dumps(meta))
    print(f"wrote {out} in {time.time() - t0:.0f} s: {json.dumps(meta)}", flush=True)


def unary(src):
    if src.startswith("batch:"):
        return make_batch_instance(make_batch_configs()[int(src.split(":")[1])])[0]
    return make_config(CONFIGS[src])[0]


def run_one(args):
    """One oracle solve; the full beliefs go to the scratch directory."""
    name, storage, scratch = args
    from threadpoolctl import threadpool_limits
    src, M, T, alpha, mode, sched, n, _ = case_list()[name]
    g32 = unary(src)
    pot = library_potential(M, T, alpha, mode)
    impl = gb.DENSE if mode == gb.SUM else gb.SPARSE
    t0 = time.time()
    with threadpool_limits(limits=1):
        state = gb.run(g32.astype(np.float64), pot, mode, n, sched, impl,
                       storage=np.float32 if storage else None)
    b = gb.beliefs(g32.astype(np.float64), state)
    tag = "f32store" if storage else "fp64"
    np.save(os.path.join(scratch, f"{name}.{tag}.npy"), b)
    print(f"{name} {tag}: {n} steps in {time.time() - t0:.0f} s", flush=True)
    return name, tag


def assemble(name, scratch):
    src, M, T, alpha, mode, sched, n, want_store = case_list()[name]
    g32 = unary(src)
    H, W, _ = g32.shape
    b = np.load(os.path.join(scratch, f"{name}.fp64.npy"))
    labels = gb.map_labels(b)
    margin = gb.top2_margin(b)
    flat_m = margin.reshape(-1)
    low = np.nonzero(flat_m <= LOW_MARGIN)[0].astype(np.int32)
    rng = np.random.default_rng(2024)
    chosen = []
    seen = set()

    def take(idx):
        for i in idx:
            i = int(i)
            if i not in seen and len(chosen) < N_SAMPLE:
                seen.add(i)
                chosen.append(i)

    take([0, W - 1, (H - 1) * W, H * W - 1])                               # corners
    for line in (np.arange(1, W - 1), (H - 1) * W + np.arange(1, W - 1),   # top, bottom rows
                 np.arange(1, H - 1) * W, np.arange(1, H - 1) * W + W - 1):  # left, right columns
        take(line[np.linspace(0, len(line) - 1, min(128, len(line))).astype(int)])
    take(np.argsort(flat_m, kind="stable")[:512])                          # closest to a tie
    extra, store = {}, {}
    store_path = os.path.join(scratch, f"{name}.f32store.npy")
    if want_store and os.path.exists(store_path):
        b32 = np.load(store_path)
        dev = np.max(np.abs(b32 - b), axis=-1).reshape(-1)
        take(np.argsort(-dev, kind="stable")[:512])                        # largest storage drift
        sure = margin > 1e-6
        extra = {"store_max_db": float(dev.max()),
                 "store_map_mismatch": int(np.sum((gb.map_labels(b32) != labels) & sure))}
        store = {"store_labels": gb.map_labels(b32).astype(np.uint8),
                 "store_low_idx": np.nonzero(gb.top2_margin(b32).reshape(-1) <= LOW_MARGIN)[0].astype(np.int32)}
        store["store_low_margin"] = gb.top2_margin(b32).reshape(-1)[store["store_low_idx"]]
    while len(chosen) < N_SAMPLE:
        take(rng.integers(0, H * W, N_SAMPLE))
    idx = np.array(chosen, dtype=np.int32)
    meta = {"case": name, "source": src, "H": H, "W": W, "M": M, "T": T, "alpha_f32": float(np.float32(alpha)),
            "mode": mode, "schedule": sched, "n": n, "impl": gb.DENSE if mode == gb.SUM else gb.SPARSE,
            "unary_sha256": hashlib.sha256(np.ascontiguousarray(g32).tobytes()).hexdigest(),
            "min_margin": float(flat_m.min()), **extra}
    out = os.path.join(HERE, f"e2e_{name}.npz")
    if store:
        # float32 is ample for a reference the GPU is held to within 1e-6
        store["store_sample_b"] = b32.reshape(H * W, M)[idx].astype(np.float32)
    np.savez_compressed(out, labels=labels.astype(np.uint8), low_idx=low, low_margin=flat_m[low],
                        sample_idx=idx, sample_b=b.reshape(H * W, M)[idx], meta=json.dumps(meta), **store)
    print(f"wrote {out}: {len(low)} pixels with margin <= {LOW_MARGIN:g}, {json.dumps(meta)}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*")
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--scratch", default=os.path.join(ROOT, "_build", "e2e_scratch"))
    ap.add_argument("--assemble", action="store_true")
    ap.add_argument("--grad", action="store_true", help="write the gradient reference only")
    a = ap.parse_args()
    if a.grad:
        write_grad_ref()
        return
    os.makedirs(a.scratch, exist_ok=True)
    cases = a.cases or list(case_list())
    if not a.assemble:
        work = [(c, s, a.scratch) for c in cases for s in ((False, True) if case_list()[c][7] else (False,))]
        # longest first (max-product 480x640 checkerboard)
        work.sort(key=lambda w: -(case_list()[w[0]][6] * (4 if case_list()[w[0]][4] == gb.MAX else 1)
                                  * (10 if "480x640" in w[0] else 1)))
        with mp.Pool(a.jobs) as pool:
            for r in pool.imap_unordered(run_one, work):
                print("done", r, flush=True)
    for c in cases:
        assemble(c, a.scratch)


if __name__ == "__main__":
    main()
