"""Pins of the oracle's multi-scale BP.

- The block unary is what a block means: on a 2 x 2 grid whose potential
  forces equal labels (T = 0, fbar = 0, the identity of Eq. 8), the exact
  marginal of every pixel is the normalised product of the four unaries,
  which is the coarse unary normalised to sum 1; partial blocks at odd edges
  keep their own children only.
- Zero levels is plain BP; the prolongation copies each parent's inbox.
- Coarse-to-fine sum-product reaches the same fixed point as plain BP (the
  schedule does not move fixed points, Sec. 2).
"""
import numpy as np
import pytest

from oracle import brute
from oracle import grid_bp as gb
from oracle import multiscale as ms


def test_block_unary_is_block_marginal():
    rng = np.random.default_rng(7)
    M = 5
    g = rng.uniform(0.05, 1.0, (2, 2, M))
    ident = gb.truncated_linear(M, 0, 1.0, 0.0)
    P = brute.joint_table(4, M, brute.grid_edges(2, 2), [ident.F] * 4, g.reshape(4, M))
    marg = brute.marginals(P)
    cu = ms.coarse_unary(g)[0, 0]
    np.testing.assert_allclose(cu / cu.sum(), marg[0], rtol=0, atol=1e-13)
    assert cu.max() == 1.0


def test_partial_blocks():
    rng = np.random.default_rng(8)
    g = rng.uniform(0.05, 1.0, (3, 5, 4))
    cu = ms.coarse_unary(g)
    assert cu.shape == (2, 3, 4)
    corner = g[2, 4] / g[2, 4].max()            # a block with one child
    np.testing.assert_allclose(cu[1, 2], corner, rtol=1e-15)
    edge = g[2, 0] * g[2, 1]                    # bottom row: two children
    np.testing.assert_allclose(cu[1, 0], edge / edge.max(), rtol=1e-15)


def test_zero_levels_is_plain_bp():
    rng = np.random.default_rng(9)
    g = rng.uniform(0.05, 1.0, (4, 5, 6))
    pot = gb.truncated_linear(6, 2, 0.7)
    np.testing.assert_array_equal(ms.run(g, pot, gb.SUM, 0, [5]), gb.run(g, pot, gb.SUM, 5))


def test_prolong_copies_parent_inbox():
    rng = np.random.default_rng(10)
    coarse = rng.uniform(size=(4, 2, 3, 5))
    fine = ms.prolong(coarse, 3, 5)
    for r in range(3):
        for c in range(5):
            np.testing.assert_array_equal(fine[:, r, c], coarse[:, r // 2, c // 2])


@pytest.mark.parametrize("schedule", [gb.SYNC, gb.CHECKERBOARD])
def test_same_fixed_point_as_plain_bp(schedule):
    rng = np.random.default_rng(11)
    H, W, M = 7, 9, 6
    g = rng.uniform(0.05, 1.0, (H, W, M))
    pot = gb.truncated_linear(M, 2, 0.8)
    n = 300 if schedule == gb.SYNC else 600
    ref = gb.beliefs(g, gb.run(g, pot, gb.SUM, n, schedule))
    got = gb.beliefs(g, ms.run(g, pot, gb.SUM, 2, [n, 40, 40], schedule))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9)


def test_storage_model_levels_are_float32():
    rng = np.random.default_rng(12)
    g = rng.uniform(0.05, 1.0, (5, 6, 8)).astype(np.float32).astype(np.float64)
    for lev in ms.pyramid(g, 2, np.float32)[1:]:
        np.testing.assert_array_equal(lev, lev.astype(np.float32).astype(np.float64))
