"""Pins of the oracle's directional sweep schedule (Sec. 6: one sweep passes
messages left, right, up and down across the lattice).

- On a chain, one sweep is the forward-backward recursion: after a single
  sweep the beliefs are the exact marginals (sum) and max-marginals (max),
  which the synchronous schedule reaches only after n - 1 iterations.  A
  scan order reversed along the pass, or a pass that read the previous
  state instead of the message just sent, fails this.
- A sweep-converged state is a fixed point of the synchronous update (the
  schedule does not move BP's fixed points, Sec. 2), and both schedules
  reach the same one.
- The vectorised pass equals message-by-message updates in scan order.

The left and right passes commute (a message sent left never reads a message
sent right: h leaves out the target's message), and so do up and down; only
horizontal-before-vertical is observable, and the message-by-message test
fixes it.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import grid_bp as gb
from tests.test_oracle_bruteforce import chain_setup, random_sparse_potential


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPLIT, gb.SPARSE])
@pytest.mark.parametrize("n,M,seed", [(2, 3, 20), (4, 4, 21), (6, 5, 22)])
def test_one_sweep_exact_on_chain_sum(vertical, impl, n, M, seed):
    rng = np.random.default_rng(seed)
    pot = random_sparse_potential(rng, M)
    g, P = chain_setup(rng, n, M, vertical, pot)
    state = gb.run(g, pot, gb.SUM, n_iters=1, schedule=gb.SWEEP, impl=impl)
    b = gb.beliefs(g, state).reshape(n, M)
    np.testing.assert_allclose(b, brute.marginals(P), rtol=0, atol=1e-12)


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPARSE])
@pytest.mark.parametrize("n,M,seed", [(3, 3, 30), (6, 5, 31)])
def test_one_sweep_exact_on_chain_max(vertical, impl, n, M, seed):
    rng = np.random.default_rng(seed)
    pot = random_sparse_potential(rng, M)          # F >= fbar: Eq. 11 is exact
    g, P = chain_setup(rng, n, M, vertical, pot)
    state = gb.run(g, pot, gb.MAX, n_iters=1, schedule=gb.SWEEP, impl=impl)
    b = gb.beliefs(g, state).reshape(n, M)
    np.testing.assert_allclose(b, brute.max_marginals(P), rtol=0, atol=1e-12)


def test_one_sync_iteration_is_not_exact_on_chain():
    """The chain pin discriminates: a Jacobi step does not finish the recursion."""
    rng = np.random.default_rng(21)
    pot = random_sparse_potential(rng, 4)
    g, P = chain_setup(rng, 4, 4, False, pot)
    b = gb.beliefs(g, gb.run(g, pot, gb.SUM, n_iters=1, schedule=gb.SYNC)).reshape(4, 4)
    assert np.max(np.abs(b - brute.marginals(P))) > 1e-4


def test_reversed_scan_is_not_exact_on_chain():
    """Visiting senders away from the pass direction reuses stale messages."""
    rng = np.random.default_rng(22)
    M, n = 5, 6
    pot = random_sparse_potential(rng, M)
    g, P = chain_setup(rng, n, M, False, pot)
    state = gb.init_messages(1, n, M)
    for o in (gb.LEFT, gb.RIGHT):
        k = gb.OPPOSITE[o]
        dc = gb.OFFSETS[o][1]
        senders = range(n - 1, 0, -1) if dc > 0 else range(0, n - 1)   # reversed
        for c in senders:
            if 0 <= c + dc < n:
                state[k, 0, c + dc] = gb.single_update(g, state, pot, gb.SUM, 0, c, o)
    b = gb.beliefs(g, state).reshape(n, M)
    assert np.max(np.abs(b - brute.marginals(P))) > 1e-4


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_pass_equals_message_by_message(mode):
    rng = np.random.default_rng(40)
    H, W, M = 3, 4, 6
    pot = gb.truncated_linear(M, 2, 0.8)
    g = rng.uniform(0.05, 1.0, (H, W, M))
    start = gb.run(g, pot, mode, n_iters=2)         # a non-uniform state
    state = start.copy()
    # the reading of Sec. 6's "left, right, up and down": the directions the
    # messages travel, in that order
    for o in (gb.LEFT, gb.RIGHT, gb.UP, gb.DOWN):
        k = gb.OPPOSITE[o]
        dr, dc = gb.OFFSETS[o]
        if dc:
            order = [(r, c) for c in (range(W) if dc > 0 else range(W - 1, -1, -1)) for r in range(H)]
        else:
            order = [(r, c) for r in (range(H) if dr > 0 else range(H - 1, -1, -1)) for c in range(W)]
        for r, c in order:
            if 0 <= r + dr < H and 0 <= c + dc < W:
                state[k, r + dr, c + dc] = gb.single_update(g, state, pot, mode, r, c, o)
    np.testing.assert_allclose(gb.sweep(g, start, pot, mode), state, rtol=0, atol=1e-15)


def test_sweep_fixed_point_is_sync_fixed_point():
    rng = np.random.default_rng(50)
    H, W, M = 5, 6, 7
    pot = gb.truncated_linear(M, 2, 0.7)
    g = rng.uniform(0.05, 1.0, (H, W, M))
    sw = gb.run(g, pot, gb.SUM, n_iters=120, schedule=gb.SWEEP)
    has = gb.has_neighbor(H, W)
    step = gb.sync_step(g, sw, pot, gb.SUM)
    assert np.max(np.abs(step - sw)[has]) < 1e-10
    sy = gb.run(g, pot, gb.SUM, n_iters=400, schedule=gb.SYNC)
    np.testing.assert_allclose(gb.beliefs(g, sw), gb.beliefs(g, sy), rtol=0, atol=1e-9)


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_sweep_forms_agree(mode):
    """Dense, split and sparse forms agree under the sweep schedule too."""
    rng = np.random.default_rng(60)
    H, W, M = 4, 5, 9
    pot = gb.truncated_linear(M, 2, 0.6)
    g = rng.uniform(0.01, 1.0, (H, W, M))
    ref = gb.run(g, pot, mode, 3, gb.SWEEP, gb.DENSE)
    for impl in (gb.SPLIT, gb.SPARSE):
        got = gb.run(g, pot, mode, 3, gb.SWEEP, impl)
        if mode == gb.MAX:
            np.testing.assert_array_equal(got, ref)
        else:
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)
