"""Pins of the factor-graph oracle (Sec. 7 higher-order factors).

- On tree-shaped factor graphs (triples sharing single variables) factor BP
  is exact: beliefs equal brute-force marginals (sum) and max-marginals
  (max), for the dense O(M^K) and the sparse O(C + M) forms;
- pairwise factors on a grid reproduce the grid oracle iteration by
  iteration (one factor-BP iteration is one synchronous grid iteration);
- dense and sparse agree (sum to 1e-12 relative, max bit for bit when
  f >= fbar on the compatible tuples).
"""
import numpy as np
import pytest

from oracle import factor_bp as fb
from oracle import grid_bp as gb


def random_type(rng, M, arity, density=0.3, below=False):
    tuples = [t for t in np.ndindex(*(M,) * arity) if rng.random() < density]
    fbar = float(rng.uniform(0.05, 0.3))
    lo = 0.0 if below else fbar
    vals = rng.uniform(lo, lo + 1.0, len(tuples))
    return fb.FactorType(arity, np.array(tuples).reshape(-1, arity), vals, fbar)


def tree_graph(rng, M):
    # triples (0,1,2), (2,3,4), (2,5,6) and a pair (4,7): a tree of factors
    types = [random_type(rng, M, 3), random_type(rng, M, 3), random_type(rng, M, 2)]
    factors = [((0, 1, 2), 0), ((2, 3, 4), 1), ((2, 5, 6), 0), ((4, 7), 2)]
    fg = fb.FactorGraph(8, M, factors, types)
    g = rng.uniform(0.05, 1.0, (8, M))
    return fg, g


@pytest.mark.parametrize("impl", [fb.DENSE, fb.SPARSE])
@pytest.mark.parametrize("mode", [fb.SUM, fb.MAX])
@pytest.mark.parametrize("M,seed", [(2, 1), (3, 2)])
def test_tree_exact(impl, mode, M, seed):
    rng = np.random.default_rng(seed)
    fg, g = tree_graph(rng, M)
    m, _ = fb.run(fg, g, mode, 8, impl)
    np.testing.assert_allclose(fb.beliefs(fg, g, m), fb.brute_marginals(fg, g, mode), rtol=0, atol=1e-12)


@pytest.mark.parametrize("mode", [fb.SUM, fb.MAX])
def test_pairwise_factors_reproduce_grid_bp(mode):
    rng = np.random.default_rng(3)
    H, W, M, T = 3, 4, 6, 2
    pot = gb.truncated_linear(M, T, 0.7)
    tuples = np.array([(x, y) for x in range(M) for y in range(M) if abs(x - y) <= T])
    ft = fb.FactorType(2, tuples, pot.F[tuples[:, 0], tuples[:, 1]], pot.fbar)
    factors = []
    for r in range(H):
        for c in range(W):
            if c + 1 < W:
                factors.append(((r * W + c, r * W + c + 1), 0))   # left, right
            if r + 1 < H:
                factors.append(((r * W + c, (r + 1) * W + c), 0))  # top, bottom
    fg = fb.FactorGraph(H * W, M, factors, [ft])
    g = rng.uniform(0.05, 1.0, (H, W, M))
    for n in (1, 2, 5):
        m, _ = fb.run(fg, g.reshape(H * W, M), mode, n)
        want = gb.beliefs(g, gb.run(g, pot, mode, n))
        np.testing.assert_allclose(fb.beliefs(fg, g.reshape(H * W, M), m).reshape(H, W, M), want, rtol=0,
                                   atol=1e-13)


@pytest.mark.parametrize("mode", [fb.SUM, fb.MAX])
def test_dense_equals_sparse_on_loopy_graph(mode):
    rng = np.random.default_rng(4)
    M = 4
    types = [random_type(rng, M, 3), random_type(rng, M, 2)]
    factors = [((0, 1, 2), 0), ((1, 2, 3), 0), ((3, 4, 0), 0), ((2, 4), 1), ((0, 3), 1)]
    fg = fb.FactorGraph(5, M, factors, types)
    g = rng.uniform(0.05, 1.0, (5, M))
    md, _ = fb.run(fg, g, mode, 6, fb.DENSE)
    ms_, _ = fb.run(fg, g, mode, 6, fb.SPARSE)
    for a in range(len(factors)):
        for i in range(len(factors[a][0])):
            if mode == fb.MAX:
                np.testing.assert_array_equal(md[a][i], ms_[a][i])
            else:
                np.testing.assert_allclose(md[a][i], ms_[a][i], rtol=1e-12, atol=0)


@pytest.mark.parametrize("M,seed", [(2, 11), (3, 12), (3, 13)])
def test_split_tree_exact_with_values_below_fbar(M, seed):
    """Max-product with compatible values below fbar: the split form (Eq. 10's
    factor analogue) gives the exact max-marginals on a tree."""
    rng = np.random.default_rng(seed)
    types = [random_type(rng, M, 3, below=True), random_type(rng, M, 3, below=True),
             random_type(rng, M, 2, below=True)]
    factors = [((0, 1, 2), 0), ((2, 3, 4), 1), ((2, 5, 6), 0), ((4, 7), 2)]
    fg = fb.FactorGraph(8, M, factors, types)
    g = rng.uniform(0.05, 1.0, (8, M))
    m, _ = fb.run(fg, g, fb.MAX, 8, fb.SPLIT)
    exact = fb.brute_marginals(fg, g, fb.MAX)
    np.testing.assert_allclose(fb.beliefs(fg, g, m), exact, atol=1e-12)


def test_split_equals_dense_bitwise_below_fbar():
    rng = np.random.default_rng(14)
    M = 4
    types = [random_type(rng, M, 3, 0.3, below=True), random_type(rng, M, 2, 0.5, below=True)]
    factors = [((0, 1, 2), 0), ((1, 2, 3), 0), ((3, 4, 0), 0), ((4, 1), 1), ((2, 4), 1)]
    fg = fb.FactorGraph(5, M, factors, types)
    g = rng.uniform(0.05, 1.0, (5, M))
    md, _ = fb.run(fg, g, fb.MAX, 6, fb.DENSE)
    msp, _ = fb.run(fg, g, fb.MAX, 6, fb.SPLIT)
    for a in range(len(factors)):
        for i in range(len(factors[a][0])):
            np.testing.assert_array_equal(md[a][i], msp[a][i])


def test_eq11_form_needs_f_at_least_fbar():
    """A pair factor that is 1 everywhere except f(0, 0) = 0: the message to
    slot 0 at label 0 is the best n_1 outside label 0.  The split form gets
    it; the fbar * max n_1 shortcut (valid only for f >= fbar) does not."""
    t = fb.FactorType(2, np.array([[0, 0]]), np.array([0.0]), 1.0)
    fg = fb.FactorGraph(2, 2, [((0, 1), 0)], [t])
    n = [[None, np.array([0.9, 0.1])]]
    assert fb.factor_message_dense(fg, 0, 0, n, fb.MAX)[0] == pytest.approx(0.1)
    assert fb.factor_message_split(fg, 0, 0, n, fb.MAX)[0] == pytest.approx(0.1)
    assert fb.factor_message_sparse(fg, 0, 0, n, fb.MAX)[0] == pytest.approx(0.9)
