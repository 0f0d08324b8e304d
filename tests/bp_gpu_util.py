"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs, and compare them."""
from __future__ import annotations

import sys

import numpy as np

from oracle import grid_bp as gb

BELIEF_TOL = 1e-5      # max |b_gpu - b_oracle| after normalisation
MAP_MARGIN = 1e-6      # MAP must match where the oracle's top-2 margin exceeds this
MSG_TOL = 1e-5         # live message entries


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(g32, M, T, alpha, fbar=None, mode="sum", schedule="sync", n_iters=5, dense=False,
            init=None, want_messages=True, fuse=True, arith="f64"):
    import torch
    from paper_1010_0012_amd.grid import Grid
    H, W, _ = g32.shape
    grid = Grid(H, W)
    grid.set_potential(M, T, alpha, fbar)
    grid.set_sync_fusion(fuse)
    grid.set_arithmetic(arith)
    g = torch.from_numpy(np.ascontiguousarray(g32)).cuda()
    grid.set_unary(g)
    if init is not None:
        grid.set_messages(torch.from_numpy(np.ascontiguousarray(init, dtype=np.float32)).cuda())
    grid.iterate(mode, n_iters, schedule, dense=dense)
    b = grid.beliefs().cpu().numpy()
    lab = grid.map_labels().cpu().numpy()
    msgs = grid.get_messages().cpu().numpy() if want_messages else None
    torch.cuda.synchronize()
    grid.close()
    return msgs, b, lab


def library_potential(M, T, alpha, fbar, mode):
    """The potential as the C ABI documents holding it: alpha and a given
    fbar are float32; sum-product uses f(d) = exp(-alpha d) in double and a
    tied fbar = f(T) in double; max-product uses the float32 table f(d) and
    fbar = float32 f(T) when tied."""
    alpha = float(np.float32(alpha))
    pot = gb.truncated_linear(M, T, alpha, None if fbar is None else float(np.float32(fbar)))
    if mode == "max":
        f32 = np.float32(np.exp(-alpha * T)) if fbar is None else np.float32(fbar)
        F = np.where(pot.compat, pot.F.astype(np.float32).astype(np.float64), float(f32))
        pot = gb.Potential(F, pot.compat, float(f32))
    return pot


def run_oracle(g32, M, T, alpha, fbar=None, mode="sum", schedule="sync", n_iters=5, impl=gb.SPARSE,
               init=None, storage=None, pot=None):
    pot = library_potential(M, T, alpha, fbar, mode) if pot is None else pot
    g = g32.astype(np.float64)
    state = gb.run(g, pot, mode, n_iters, schedule, impl,
                   inbox=None if init is None else init.astype(np.float64), storage=storage)
    b = gb.beliefs(g, state)
    return state, b, gb.map_labels(b)


STORAGE_TOL = 1e-6     # GPU vs the oracle's float32-storage model

# Cases on which the oracle's own float32-storage model (FP64 arithmetic,
# every message rounded once to float32 when it is stored) already misses
# the FP64 bar: no implementation that stores float32 messages can meet it
# there.  Max-product does not contract perturbations (each message takes its
# winning label's error unchanged and h multiplies three of them), and
# sum-product with fbar = 0 stores zeros and denormals.  Only these cases are
# judged against the storage model alone; check_against asserts for each
# that the storage model really misses the bar, and prints the GPU's FP64
# figures as not meeting it.  Every other case is held to the bar unchanged:
# beliefs and messages within 1e-5 of FP64, MAP equal where the FP64 margin
# exceeds 1e-6.  Keys are the tags the tests pass.
STORAGE_LIMITED = {
    # f32-storage model alone: messages 1.5e-5 from FP64 (beliefs 5.2e-6)
    "fbar zero": "sum-product with fbar = 0 stores zeros and denormals",
    # max-product synchronous BP oscillates on this grid (beliefs change by
    # up to 0.99 between consecutive iterations), so one float32 rounding
    # per stored message moves the 50-iteration beliefs by 3.6e-2
    "stereo288x384_max_sync": "max-product, oscillating synchronous iterations",
    # f32-storage model alone: beliefs 1.7e-5 from FP64 after 100 passes
    "stereo288x384_max_checkerboard": "max-product does not contract rounding",
    # f32-storage model alone: beliefs 4.9e-5 from FP64 after 100 iterations
    "stereo480x640_max_sync": "max-product does not contract rounding",
    # f32-storage model alone: beliefs 1.9e-5 from FP64 after 30 iterations
    # (403 x 493, M = 128, T = 3; the smallest top-two margin is 6.8e-6)
    "batch32_5_sum_sync": "sum-product, M = 128, a weakly damped instance",
}

# (tag, max|db| vs FP64, MAP mismatches vs FP64 at margin 1e-6, storage-only
# max|db|) of every storage-limited case met in this session.
STORAGE_LIMITED_SEEN = []


def check(tag, gpu, g32, M, T, alpha, fbar, mode, schedule, n_iters, impl=gb.SPARSE, init=None,
          check_msgs=True, pot=None):
    """Compare a GPU result with the FP64 oracle and with the oracle's
    float32-storage model (FP64 arithmetic, each stored message rounded once
    to float32), which the GPU's double arithmetic reproduces up to rare
    one-ulp differences; the rule is check_against's."""
    ref = run_oracle(g32, M, T, alpha, fbar, mode, schedule, n_iters, impl, init, pot=pot)
    ref32 = run_oracle(g32, M, T, alpha, fbar, mode, schedule, n_iters, impl, init, storage=np.float32, pot=pot)
    check_against(tag, gpu, g32, ref, ref32, check_msgs)


def oracle_result(g32, state):
    """(state, beliefs, MAP) of an oracle state on the unary g32."""
    b = gb.beliefs(g32.astype(np.float64), state)
    return state, b, gb.map_labels(b)


def storage_misses_bar(ref, ref32, has):
    """Whether the float32-storage model itself misses the FP64 bar, and by
    how much (max|db|, max|dm| over live messages, MAP mismatches where the
    FP64 margin exceeds 1e-6)."""
    dev_b = float(np.max(np.abs(ref32[1] - ref[1])))
    dev_m = float(np.max(np.abs(ref32[0] - ref[0])[has])) if has.any() else 0.0
    sure = gb.top2_margin(ref[1]) > MAP_MARGIN
    flips = int(np.sum((ref32[2] != ref[2]) & sure))
    return (dev_b > BELIEF_TOL or dev_m > MSG_TOL or flips > 0), dev_b, dev_m, flips


def check_against(tag, gpu, g32, ref, ref32, check_msgs=True):
    """The parity rule for given FP64 and float32-storage oracle results.

    Always: within 1e-6 of the storage model (beliefs, live messages) and
    the same MAP labels where its margin exceeds 1e-6.  Then, unless the
    case is named in STORAGE_LIMITED: the FP64 bar itself.  A named case must
    be one where the storage model misses the FP64 bar; its FP64 figures are
    reported as not meeting it."""
    compare(tag + " [f32-storage model]", gpu, ref32, belief_tol=STORAGE_TOL, msg_tol=STORAGE_TOL,
            check_msgs=check_msgs)
    H, W, _ = g32.shape
    has = gb.has_neighbor(H, W)
    missed, dev_b, dev_m, flips = storage_misses_bar(ref, ref32, has)
    if tag not in STORAGE_LIMITED:
        if missed:
            say(f"{tag}: the float32-storage model itself misses the FP64 bar (max|db|={dev_b:.2e}, "
                f"max|dm|={dev_m:.2e}, MAP flips={flips}); if the GPU misses it too, name the case in "
                f"STORAGE_LIMITED")
        compare(tag + " [FP64]", gpu, ref, check_msgs=check_msgs)
        return
    assert missed, (f"{tag} is named storage-limited, but the float32-storage model meets the FP64 bar "
                    f"(max|db|={dev_b:.2e}, max|dm|={dev_m:.2e}); remove it from STORAGE_LIMITED")
    msgs, b, lab = gpu
    err_b = float(np.max(np.abs(b - ref[1])))
    sure = gb.top2_margin(ref[1]) > MAP_MARGIN
    bad = int(np.sum((lab != ref[2]) & sure))
    say(f"{tag} [FP64, storage-limited: {STORAGE_LIMITED[tag]}]: FP64 bar NOT met by float32 storage: "
        f"GPU max|db|={err_b:.2e}, MAP mismatches={bad}; storage model alone max|db|={dev_b:.2e}, "
        f"max|dm|={dev_m:.2e}, MAP flips={flips}")
    STORAGE_LIMITED_SEEN.append((tag, err_b, bad, dev_b))
    # the GPU is no further from FP64 than the storage format allows
    assert err_b <= dev_b + STORAGE_TOL, (tag, err_b, dev_b)


def compare(tag, gpu, ref, belief_tol=BELIEF_TOL, msg_tol=MSG_TOL, check_msgs=True, map_margin=MAP_MARGIN):
    """Assert the GPU result (msgs, beliefs, labels) matches the oracle's."""
    msgs, b, lab = gpu
    state, b_ref, lab_ref = ref
    H, W, M = b_ref.shape
    err_b = float(np.max(np.abs(b - b_ref)))
    sure = gb.top2_margin(b_ref) > map_margin
    bad = (lab != lab_ref) & sure
    line = f"{tag}: max|db|={err_b:.2e} MAP mismatches={int(bad.sum())}/{int(sure.sum())}"
    if check_msgs and msgs is not None:
        has = gb.has_neighbor(H, W)
        err_m = float(np.max(np.abs(msgs - state)[has])) if has.any() else 0.0
        line += f" max|dm|={err_m:.2e}"
        assert err_m <= msg_tol, line
    say(line)
    assert err_b <= belief_tol, line
    if bad.any():
        idx = np.argwhere(bad)[:5]
        detail = [(tuple(i), int(lab[tuple(i)]), int(lab_ref[tuple(i)]),
                   float(gb.top2_margin(b_ref)[tuple(i)])) for i in idx]
        raise AssertionError(f"{line}; first mismatches (pixel, gpu, oracle, margin): {detail}")
    # labels are the argmax of the returned float32 beliefs (lowest index on ties)
    np.testing.assert_array_equal(lab, np.argmax(b, axis=-1))
