"""Pin the FP64 oracle with identities the paper and the mathematics fix.

- Eq. 7 (sparse) = Eq. 6 (split) = Eq. 2 (dense), every iteration (Sec. 4:
  the trick is exact); identical MAP labels (Sec. 6).
- Eq. 11 = Eq. 9 whenever f >= fbar, and not otherwise; Eq. 10 always (Sec. 5).
- Normalisation, closed forms, the checkerboard/sync interleave, metamorphic
  symmetries and lower bounds.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import grid_bp as gb
from synth_mrf import make_stereo, random_unary

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_case(seed=0, H=6, W=7, M=9):
    g32, D, _, _ = make_stereo(H, W, M, 0.05, 4.0, "rectangles", seed)
    return g32.astype(np.float64), D


@pytest.mark.parametrize("fbar", [None, 0.3, 0.0])
def test_sum_forms_agree_every_iteration(fbar):
    g, _ = small_case()
    pot = gb.truncated_linear(9, 2, 0.8, fbar)
    s_dense = s_split = s_sparse = gb.init_messages(*g.shape)
    for _ in range(8):
        s_dense = gb.sync_step(g, s_dense, pot, gb.SUM, gb.DENSE)
        s_split = gb.sync_step(g, s_split, pot, gb.SUM, gb.SPLIT)
        s_sparse = gb.sync_step(g, s_sparse, pot, gb.SUM, gb.SPARSE)
        np.testing.assert_allclose(s_split, s_dense, rtol=1e-12, atol=0)
        np.testing.assert_allclose(s_sparse, s_dense, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(gb.map_labels(gb.beliefs(g, s_sparse)),
                                  gb.map_labels(gb.beliefs(g, s_dense)))


def test_sum_forms_agree_checkerboard():
    g, _ = small_case(1, 5, 8, 7)
    pot = gb.truncated_linear(7, 1, 1.3)
    a = gb.run(g, pot, gb.SUM, 9, gb.CHECKERBOARD, gb.DENSE)
    b = gb.run(g, pot, gb.SUM, 9, gb.CHECKERBOARD, gb.SPARSE)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=0)


def test_max_sparse_equals_dense_bitwise_when_f_ge_fbar():
    g, _ = small_case(2)
    pot = gb.truncated_linear(9, 2, 0.8)      # fbar = exp(-alpha T) <= f
    for sched in (gb.SYNC, gb.CHECKERBOARD):
        a = gb.run(g, pot, gb.MAX, 7, sched, gb.DENSE)
        b = gb.run(g, pot, gb.MAX, 7, sched, gb.SPARSE)
        c = gb.run(g, pot, gb.MAX, 7, sched, gb.SPLIT)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)


def test_max_sparse_needs_f_ge_fbar():
    """With fbar above some f (violating Sec. 5's assumption) Eq. 11 differs from
    Eq. 9, while Eq. 10 still equals it."""
    g, _ = small_case(3)
    pot = gb.truncated_linear(9, 2, 0.8, fbar=0.9)
    a = gb.run(g, pot, gb.MAX, 3, gb.SYNC, gb.DENSE)
    b = gb.run(g, pot, gb.MAX, 3, gb.SYNC, gb.SPARSE)
    c = gb.run(g, pot, gb.MAX, 3, gb.SYNC, gb.SPLIT)
    np.testing.assert_array_equal(a, c)
    assert np.max(np.abs(a - b)) > 1e-3


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_messages_normalised(mode):
    g, _ = small_case(4)
    pot = gb.truncated_linear(9, 2, 0.8)
    state = gb.run(g, pot, mode, 5)
    np.testing.assert_allclose(gb.message_sums(state), 1.0, atol=1e-13)


def test_closed_form_flat_potential():
    """alpha = 0, fbar = 1: F is all ones, so every message is uniform after one
    iteration and the beliefs are g / sum g."""
    g, _ = small_case(5)
    pot = gb.truncated_linear(9, 2, 0.0, fbar=1.0)
    state = gb.run(g, pot, gb.SUM, 1)
    np.testing.assert_allclose(state, 1.0 / 9, atol=1e-15)
    np.testing.assert_allclose(gb.beliefs(g, state), g / g.sum(-1, keepdims=True), atol=1e-15)


def test_closed_form_no_iterations():
    g, _ = small_case(6)
    b = gb.beliefs(g, gb.init_messages(*g.shape))
    np.testing.assert_allclose(b, g / g.sum(-1, keepdims=True), atol=1e-15)


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                key, rhs = line.split("=", 1)
                vals[key.strip()] = [float(Fraction(v.strip())) for v in rhs.split(",")]
    return vals


def test_two_node_hand_worked_example():
    """A 1 x 2 grid, M = 3, worked by hand (tests/golden/two_node_hand.txt)."""
    v = read_golden("two_node_hand.txt")
    g = np.array([[v["g1"], v["g2"]]], dtype=np.float64)
    pot = gb.truncated_linear(3, 1, np.log(2.0))
    for mode, key in ((gb.SUM, "b1_sum"), (gb.MAX, "b1_max")):
        for impl in (gb.DENSE, gb.SPLIT, gb.SPARSE):
            b = gb.beliefs(g, gb.run(g, pot, mode, 1, impl=impl))
            np.testing.assert_allclose(b[0, 0], v[key], rtol=1e-14)
    b2 = gb.beliefs(g, gb.run(g, pot, gb.SUM, 1))
    np.testing.assert_allclose(b2[0, 1], v["b2_sum"], rtol=1e-14)
    assert gb.map_labels(gb.beliefs(g, gb.run(g, pot, gb.MAX, 1)))[0, 0] == v["map1"][0]


def test_identity_potential_chain():
    """T = 0, fbar = 0 (Eq. 8 with Nbd(x) = {x}): F = I, so on a chain every
    belief is proportional to the product of all unaries."""
    rng = np.random.default_rng(0)
    n, M = 6, 5
    g = rng.uniform(0.1, 1.0, (1, n, M))
    pot = gb.truncated_linear(M, 0, 1.0, fbar=0.0)
    b = gb.beliefs(g, gb.run(g, pot, gb.SUM, n))
    prod = np.prod(g[0], axis=0)
    np.testing.assert_allclose(b[0], np.broadcast_to(prod / prod.sum(), (n, M)), atol=1e-14)


def test_fbar_zero_is_eq8():
    """fbar = 0: Eq. 7 reduces to Eq. 8, the sum over compatible states only."""
    rng = np.random.default_rng(1)
    M, T = 8, 2
    pot = gb.truncated_linear(M, T, 0.6, fbar=0.0)
    h = rng.uniform(0, 1, (5, M))
    eq8 = np.zeros((5, M))
    for y in range(M):
        for x in range(max(0, y - T), min(M, y + T + 1)):
            eq8[:, y] += np.exp(-0.6 * abs(x - y)) * h[:, x]
    np.testing.assert_allclose(gb.message_sparse_sum(h, pot), eq8, rtol=1e-14)


def test_sparse_sum_matches_explicit_double_loop():
    """Eq. 7 with an explicit O(M^2) double loop over (x_j, x_i) for a random
    sparse-compatible asymmetric potential."""
    rng = np.random.default_rng(2)
    M = 7
    compat = rng.random((M, M)) < 0.3
    F = np.where(compat, rng.uniform(0, 2, (M, M)), 0.25)
    pot = gb.Potential(F, compat, 0.25)
    h = rng.uniform(0, 1, (3, M))
    ref = np.zeros((3, M))
    for xj in range(M):
        for xi in range(M):
            ref[:, xj] += F[xi, xj] * h[:, xi]
    np.testing.assert_allclose(gb.message_sparse_sum(h, pot), ref, rtol=1e-13)
    np.testing.assert_allclose(gb.message_split_sum(h, pot), ref, rtol=1e-13)


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_checkerboard_interleaves_sync(mode):
    """After n passes, senders of colour (n-1) mod 2 hold the sync state m^n and
    the others m^(n-1) (the two colours' updates are independent chains)."""
    g, _ = small_case(7, 7, 6, 9)
    H, W, M = g.shape
    pot = gb.truncated_linear(M, 2, 0.8)
    n = 5
    _, sync_states = gb.run(g, pot, mode, n, gb.SYNC, record=True)
    cb = gb.run(g, pot, mode, n, gb.CHECKERBOARD)
    has = gb.has_neighbor(H, W)
    for k in gb.DIRS:
        dr, dc = gb.OFFSETS[k]
        for r in range(H):
            for c in range(W):
                if not has[k, r, c]:
                    continue
                sender_colour = (r + dr + c + dc) % 2
                ref = sync_states[n] if sender_colour == (n - 1) % 2 else sync_states[n - 1]
                np.testing.assert_array_equal(cb[k, r, c], ref[k, r, c])


def test_transpose_symmetry():
    g, _ = small_case(8, 5, 7, 6)
    pot = gb.truncated_linear(6, 1, 0.9)
    gt = np.ascontiguousarray(np.transpose(g, (1, 0, 2)))
    s = gb.run(g, pot, gb.SUM, 6)
    st = gb.run(gt, pot, gb.SUM, 6)
    relabel = {gb.LEFT: gb.UP, gb.RIGHT: gb.DOWN, gb.UP: gb.LEFT, gb.DOWN: gb.RIGHT}
    for k in gb.DIRS:
        np.testing.assert_allclose(np.transpose(s[k], (1, 0, 2)), st[relabel[k]], rtol=1e-12)


def test_flip_symmetry():
    g, _ = small_case(9, 5, 7, 6)
    pot = gb.truncated_linear(6, 1, 0.9)
    s = gb.run(g, pot, gb.MAX, 6)
    sf = gb.run(g[:, ::-1].copy(), pot, gb.MAX, 6)
    np.testing.assert_allclose(s[gb.LEFT][:, ::-1], sf[gb.RIGHT], rtol=1e-12)
    np.testing.assert_allclose(s[gb.UP][:, ::-1], sf[gb.UP], rtol=1e-12)


def test_label_reversal_and_scaling():
    g, _ = small_case(10, 4, 5, 8)
    pot = gb.truncated_linear(8, 2, 0.5)
    b = gb.beliefs(g, gb.run(g, pot, gb.SUM, 5))
    br = gb.beliefs(g[..., ::-1].copy(), gb.run(g[..., ::-1].copy(), pot, gb.SUM, 5))
    np.testing.assert_allclose(b[..., ::-1], br, rtol=1e-12)
    bs = gb.beliefs(3.7 * g, gb.run(3.7 * g, pot, gb.SUM, 5))
    np.testing.assert_allclose(bs, b, rtol=1e-12)


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_lower_bounds(mode):
    """With f <= 1: every message entry >= fbar / M; with g <= 1 every belief
    >= g_min * (fbar / M)^4."""
    g = random_unary(6, 6, 10, 11, low=1e-3).astype(np.float64)
    pot = gb.truncated_linear(10, 2, 1.5)
    state = gb.run(g, pot, mode, 6)
    has = gb.has_neighbor(6, 6)
    assert np.min(state[has]) >= pot.fbar / 10 * (1 - 1e-12)
    assert np.min(gb.beliefs(g, state)) >= g.min() * (pot.fbar / 10) ** 4


def test_single_update_matches_grid_step():
    g, _ = small_case(11)
    pot = gb.truncated_linear(9, 2, 0.8)
    s0 = gb.run(g, pot, gb.SUM, 3)
    s1 = gb.sync_step(g, s0, pot, gb.SUM)
    H, W, _ = g.shape
    for (r, c, o) in [(0, 0, gb.RIGHT), (2, 3, gb.UP), (5, 6, gb.LEFT), (4, 0, gb.DOWN)]:
        m = gb.single_update(g, s0, pot, gb.SUM, r, c, o)
        dr, dc = gb.OFFSETS[o]
        np.testing.assert_allclose(m, s1[gb.OPPOSITE[o], r + dr, c + dc], rtol=1e-13)
    np.testing.assert_allclose(gb.single_belief(g, s1, 2, 2), gb.beliefs(g, s1)[2, 2], rtol=1e-14)
