"""Pin the FP64 oracle to exhaustive enumeration where BP is exact (trees).

Chains run through the grid oracle itself (as 1 x n and n x 1 grids, so both
the horizontal and the vertical message paths are covered); general trees run
through the edge-list oracle, which in turn cross-checks the grid oracle's
indexing on loopy grids.
"""
import numpy as np
import pytest

from oracle import brute, graph_bp
from oracle import grid_bp as gb


def random_sparse_potential(rng, M, density=0.4, fbar=0.15, asymmetric=True, floor_fbar=True):
    """A random sparse-compatible potential: compatible pairs get values >= fbar
    (so Eq. 11 also applies), every other pair gets fbar."""
    compat = rng.random((M, M)) < density
    np.fill_diagonal(compat, True)
    if not asymmetric:
        compat = compat | compat.T
    lo = fbar if floor_fbar else 0.0
    vals = rng.uniform(lo, lo + 1.0, (M, M))
    if not asymmetric:
        vals = np.triu(vals) + np.triu(vals, 1).T
    F = np.where(compat, vals, fbar)
    return gb.Potential(F, compat, fbar)


def chain_setup(rng, n, M, vertical, pot):
    g = rng.uniform(0.05, 1.0, (n, M))
    H, W = (n, 1) if vertical else (1, n)
    edges = brute.grid_edges(H, W)
    P = brute.joint_table(n, M, edges, [pot.F] * len(edges), g)
    return g.reshape(H, W, M), P


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPLIT, gb.SPARSE])
@pytest.mark.parametrize("n,M,seed", [(2, 3, 0), (4, 4, 1), (6, 5, 2), (5, 5, 3)])
def test_chain_sum_marginals(vertical, impl, n, M, seed):
    rng = np.random.default_rng(seed)
    pot = random_sparse_potential(rng, M)
    g, P = chain_setup(rng, n, M, vertical, pot)
    state = gb.run(g, pot, gb.SUM, n_iters=n - 1 + 2, impl=impl)
    b = gb.beliefs(g, state).reshape(n, M)
    np.testing.assert_allclose(b, brute.marginals(P), rtol=0, atol=1e-12)


@pytest.mark.parametrize("vertical", [False, True])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPLIT, gb.SPARSE])
@pytest.mark.parametrize("n,M,seed", [(3, 3, 10), (5, 4, 11), (6, 5, 12)])
def test_chain_max_marginals_and_map(vertical, impl, n, M, seed):
    rng = np.random.default_rng(seed)
    pot = random_sparse_potential(rng, M)          # F >= fbar: Eq. 11 is exact
    g, P = chain_setup(rng, n, M, vertical, pot)
    state = gb.run(g, pot, gb.MAX, n_iters=n + 1, impl=impl)
    b = gb.beliefs(g, state).reshape(n, M)
    np.testing.assert_allclose(b, brute.max_marginals(P), rtol=0, atol=1e-12)
    x_map, unique = brute.map_state(P)
    assert unique
    np.testing.assert_array_equal(gb.map_labels(b), x_map)


@pytest.mark.parametrize("seed", range(4))
def test_chain_truncated_linear(seed):
    """The stereo potential on a chain, all three forms, both modes."""
    rng = np.random.default_rng(100 + seed)
    n, M, T = 5, 5, 1
    pot = gb.truncated_linear(M, T, alpha=0.7)
    g, P = chain_setup(rng, n, M, False, pot)
    for impl in (gb.DENSE, gb.SPLIT, gb.SPARSE):
        b = gb.beliefs(g, gb.run(g, pot, gb.SUM, n + 1, impl=impl)).reshape(n, M)
        np.testing.assert_allclose(b, brute.marginals(P), atol=1e-12)
        bm = gb.beliefs(g, gb.run(g, pot, gb.MAX, n + 1, impl=impl)).reshape(n, M)
        np.testing.assert_allclose(bm, brute.max_marginals(P), atol=1e-12)


def random_tree(rng, n):
    return [(int(rng.integers(0, i)), i) for i in range(1, n)]


@pytest.mark.parametrize("seed", range(6))
def test_tree_graph_bp(seed):
    rng = np.random.default_rng(200 + seed)
    n, M = 7, 3
    edges = random_tree(rng, n)
    # orient half the edges the other way to exercise the factor orientation
    edges = [(b, a) if rng.random() < 0.5 else (a, b) for a, b in edges]
    F_list = [random_sparse_potential(rng, M).F for _ in edges]
    g = rng.uniform(0.05, 1.0, (n, M))
    mrf = graph_bp.PairwiseMRF(n, M, edges, F_list, g)
    P = brute.joint_table(n, M, edges, F_list, g)
    b = graph_bp.beliefs(mrf, graph_bp.run_bp(mrf, "sum", n_iters=n))
    np.testing.assert_allclose(b, brute.marginals(P), atol=1e-12)
    bm = graph_bp.beliefs(mrf, graph_bp.run_bp(mrf, "max", n_iters=n))
    np.testing.assert_allclose(bm, brute.max_marginals(P), atol=1e-12)


@pytest.mark.parametrize("mode", [gb.SUM, gb.MAX])
@pytest.mark.parametrize("impl", [gb.DENSE, gb.SPARSE])
def test_grid_matches_graph_bp_on_loopy_grid(mode, impl):
    """The vectorised grid oracle and the per-edge oracle agree on a loopy grid
    with an asymmetric potential (pins the 2-D neighbour indexing)."""
    rng = np.random.default_rng(7)
    H, W, M = 3, 4, 4
    pot = random_sparse_potential(rng, M)
    g = rng.uniform(0.05, 1.0, (H, W, M))
    edges = brute.grid_edges(H, W)
    mrf = graph_bp.PairwiseMRF(H * W, M, edges, [pot.F] * len(edges), g.reshape(-1, M))
    n = 6
    msgs = graph_bp.run_bp(mrf, mode, n)
    state = gb.run(g, pot, mode, n, impl=impl)
    for p in range(H * W):
        r, c = divmod(p, W)
        for k in gb.DIRS:
            dr, dc = gb.OFFSETS[k]
            rr, cc = r + dr, c + dc
            if 0 <= rr < H and 0 <= cc < W:
                np.testing.assert_allclose(state[k, r, c], msgs[(rr * W + cc, p)], atol=1e-13)
    np.testing.assert_allclose(gb.beliefs(g, state).reshape(-1, M),
                               graph_bp.beliefs(mrf, msgs), atol=1e-13)


def test_brute_force_itself_on_two_nodes():
    """Enumeration agrees with an explicit double loop on two nodes."""
    rng = np.random.default_rng(3)
    M = 4
    F = rng.uniform(0.1, 1, (M, M))
    g = rng.uniform(0.1, 1, (2, M))
    P = brute.joint_table(2, M, [(0, 1)], [F], g)
    for x0 in range(M):
        for x1 in range(M):
            assert P[x0, x1] == pytest.approx(g[0, x0] * g[1, x1] * F[x0, x1], rel=1e-15)
    P_rev = brute.joint_table(2, M, [(1, 0)], [F], g)
    for x0 in range(M):
        for x1 in range(M):
            assert P_rev[x0, x1] == pytest.approx(g[0, x0] * g[1, x1] * F[x1, x0], rel=1e-15)
