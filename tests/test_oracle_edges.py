"""Pins of the oracle's general sparse-compatible potentials (Sec. 4: a
potential per edge with its own fbar and neighbourhood, not necessarily a
function of x_i - x_j; Sec. 5: Eq. 10 when f >= fbar fails).

- chains with a different random non-difference potential on every edge
  against brute-force marginals and max-marginals, horizontal and vertical;
  including potentials with compatible pairs below fbar, where Eq. 10 (the
  split form) stays exact (Eq. 11 is checked only where f >= fbar);
- a loopy grid with per-edge types against the independent edge-list BP;
- a single type everywhere equals the plain potential.
"""
import numpy as np
import pytest

from oracle import brute, graph_bp
from oracle import grid_bp as gb
from tests.test_oracle_bruteforce import random_sparse_potential


def random_types(rng, M, k, below_fbar=False):
    """k random sparse-compatible potentials; with below_fbar some compatible
    pairs take values under fbar."""
    out = []
    for _ in range(k):
        fbar = float(rng.uniform(0.05, 0.4))
        p = random_sparse_potential(rng, M, density=0.3, fbar=fbar, floor_fbar=not below_fbar)
        out.append(p)
    return out


def chain(rng, n, M, vertical, types):
    H, W = (n, 1) if vertical else (1, n)
    th = rng.integers(0, len(types), (H, max(W - 1, 0)))
    tv = rng.integers(0, len(types), (max(H - 1, 0), W))
    pot = gb.EdgePotentials(types, th, tv)
    g = rng.uniform(0.05, 1.0, (H, W, M))
    edges = brute.grid_edges(H, W)
    F_list = []
    for a, b in edges:
        (ra, ca), (rb, cb) = divmod(a, W), divmod(b, W)
        F_list.append(types[int(th[ra, ca] if ra == rb else tv[ra, ca])].F)
    P = brute.joint_table(n, M, edges, F_list, g.reshape(n, M))
    return g, pot, P


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPLIT, gb.SPARSE])
@pytest.mark.parametrize("n,M,seed", [(4, 4, 70), (6, 5, 71)])
def test_per_edge_chain_sum(vertical, impl, n, M, seed):
    rng = np.random.default_rng(seed)
    g, pot, P = chain(rng, n, M, vertical, random_types(rng, M, 3))
    for schedule, iters in ((gb.SYNC, n + 1), (gb.SWEEP, 1)):
        st = gb.run(g, pot, gb.SUM, iters, schedule, impl)
        np.testing.assert_allclose(gb.beliefs(g, st).reshape(n, M), brute.marginals(P), rtol=0, atol=1e-12)


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("below", [False, True])
@pytest.mark.parametrize("n,M,seed", [(4, 4, 80), (6, 5, 81)])
def test_per_edge_chain_max(vertical, below, n, M, seed):
    rng = np.random.default_rng(seed)
    g, pot, P = chain(rng, n, M, vertical, random_types(rng, M, 3, below_fbar=below))
    want = brute.max_marginals(P)
    for schedule, iters in ((gb.SYNC, n + 1), (gb.SWEEP, 1)):   # one sweep is exact on a chain
        for impl in (gb.DENSE, gb.SPLIT):           # Eq. 9 and Eq. 10: exact for any fbar
            st = gb.run(g, pot, gb.MAX, iters, schedule, impl)
            np.testing.assert_allclose(gb.beliefs(g, st).reshape(n, M), want, rtol=0, atol=1e-12)
        if not below:                                # Eq. 11 needs f >= fbar (Sec. 5)
            st = gb.run(g, pot, gb.MAX, iters, schedule, gb.SPARSE)
            np.testing.assert_allclose(gb.beliefs(g, st).reshape(n, M), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_per_edge_grid_matches_edge_list(mode):
    rng = np.random.default_rng(90)
    H, W, M = 4, 5, 5
    types = random_types(rng, M, 3, below_fbar=(mode == gb.MAX))
    th = rng.integers(0, 3, (H, W - 1))
    tv = rng.integers(0, 3, (H - 1, W))
    pot = gb.EdgePotentials(types, th, tv)
    g = rng.uniform(0.05, 1.0, (H, W, M))
    edges = brute.grid_edges(H, W)
    F_list = []
    for a, b in edges:
        (ra, ca), (rb, cb) = divmod(a, W), divmod(b, W)
        F_list.append(types[int(th[ra, ca] if ra == rb else tv[ra, ca])].F)
    mrf = graph_bp.PairwiseMRF(H * W, M, edges, F_list, g.reshape(H * W, M))
    want = graph_bp.beliefs(mrf, graph_bp.run_bp(mrf, mode, 6)).reshape(H, W, M)
    impl = gb.SPLIT if mode == gb.MAX else gb.SPARSE
    got = gb.beliefs(g, gb.run(g, pot, mode, 6, gb.SYNC, impl))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_single_type_equals_plain_potential():
    rng = np.random.default_rng(95)
    H, W, M = 3, 4, 7
    p = gb.truncated_linear(M, 2, 0.6)
    pot = gb.EdgePotentials([p], np.zeros((H, W - 1)), np.zeros((H - 1, W)))
    g = rng.uniform(0.05, 1.0, (H, W, M))
    for schedule in (gb.SYNC, gb.CHECKERBOARD, gb.SWEEP):
        np.testing.assert_allclose(gb.run(g, pot, gb.SUM, 3, schedule), gb.run(g, p, gb.SUM, 3, schedule),
                                   rtol=1e-14, atol=0)  # row selection changes NumPy's summation order


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
def test_single_update_per_edge_matches_step(mode):
    """Message-by-message (used for sampled checks) equals the vectorised step."""
    rng = np.random.default_rng(97)
    H, W, M = 3, 4, 6
    types = random_types(rng, M, 3)
    pot = gb.EdgePotentials(types, rng.integers(0, 3, (H, W - 1)), rng.integers(0, 3, (H - 1, W)))
    g = rng.uniform(0.05, 1.0, (H, W, M))
    s0 = gb.run(g, pot, mode, 2)
    s1 = gb.sync_step(g, s0, pot, mode)
    for r in range(H):
        for c in range(W):
            for o in gb.DIRS:
                dr, dc = gb.OFFSETS[o]
                if 0 <= r + dr < H and 0 <= c + dc < W:
                    np.testing.assert_allclose(gb.single_update(g, s0, pot, mode, r, c, o),
                                               s1[gb.OPPOSITE[o], r + dr, c + dc], rtol=1e-13, atol=0)
