"""Pins of the oracle's readout helpers (Eq. 3 beliefs, the MAP labels of
the Sec. 6 disparity map, and the top-two margin that decides where the GPU's
MAP labels must equal the oracle's)."""
import numpy as np
import pytest

from oracle import grid_bp as gb


def margin_brute(row):
    """Largest entry minus the largest of the others (one copy of the
    maximum removed, so a tie gives 0), by a plain loop."""
    row = [float(v) for v in row]
    if len(row) < 2:
        return float("inf")
    i = max(range(len(row)), key=lambda k: row[k])
    rest = row[:i] + row[i + 1:]
    return row[i] - max(rest)


def test_top2_margin_examples():
    b = np.array([[0.1, 0.5, 0.4], [0.3, 0.3, 0.4], [0.5, 0.5, 0.0], [1.0, 0.0, 0.0]])
    np.testing.assert_allclose(gb.top2_margin(b), [0.1, 0.1, 0.0, 1.0], rtol=0, atol=1e-15)
    assert gb.top2_margin(np.ones((2, 3, 1)))[1, 2] == np.inf


@pytest.mark.parametrize("M", [2, 3, 7, 64])
def test_top2_margin_brute_force(M):
    rng = np.random.default_rng(M)
    b = rng.random((5, 6, M))
    b[0, 0, :2] = 0.75                      # an exact tie at the top
    b[1, 1] = 0.0
    b[1, 1, M - 1] = 1.0                    # a single nonzero entry
    got = gb.top2_margin(b)
    assert got.shape == (5, 6)
    for r in range(5):
        for c in range(6):
            assert got[r, c] == margin_brute(b[r, c])
    assert got[0, 0] == 0.0 or b[0, 0].max() > 0.75


def test_map_labels_lowest_index_on_ties():
    b = np.array([[[0.2, 0.4, 0.4], [0.5, 0.25, 0.25], [0.1, 0.1, 0.8]]])
    np.testing.assert_array_equal(gb.map_labels(b), [[1, 0, 2]])
