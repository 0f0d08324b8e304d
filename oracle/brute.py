"""Exhaustive inference on tiny pairwise MRFs (Eq. 1), FP64.

TEST INFRASTRUCTURE ONLY: never imported by the product path.

Enumerates every joint state, so it is limited to M**n of a few hundred
thousand.  It is the ground truth BP must reproduce on trees: sum-product
beliefs equal the exact marginals and max-product beliefs (normalised) equal
the exact max-marginals.
"""
from __future__ import annotations

import itertools

import numpy as np


def joint_table(n, M, edges, F_list, g):
    """Unnormalised joint P(x) of Eq. 1 as an array of shape (M,) * n.

    edges[e] = (a, b) uses the factor F_list[e][x_a, x_b]; g is [n, M].
    """
    g = np.asarray(g, dtype=np.float64)
    P = np.ones((M,) * n, dtype=np.float64)
    for i in range(n):
        shape = [1] * n
        shape[i] = M
        P = P * g[i].reshape(shape)
    for (a, b), F in zip(edges, F_list):
        F = np.asarray(F, dtype=np.float64)
        if a < b:
            shape = [1] * n
            shape[a], shape[b] = M, M
            P = P * F.reshape(shape)
        else:
            shape = [1] * n
            shape[b], shape[a] = M, M
            P = P * F.T.reshape(shape)
    return P


def marginals(P):
    """Exact single-node marginals, [n, M]."""
    n = P.ndim
    Z = P.sum()
    return np.stack([P.sum(axis=tuple(j for j in range(n) if j != i)) / Z for i in range(n)])


def max_marginals(P):
    """Exact max-marginals max_{x: x_i = s} P(x), normalised per node to sum 1."""
    n = P.ndim
    out = []
    for i in range(n):
        mm = P.max(axis=tuple(j for j in range(n) if j != i))
        out.append(mm / mm.sum())
    return np.stack(out)


def map_state(P):
    """The jointly most probable state and whether it is unique."""
    flat = P.ravel()
    best = flat.max()
    winners = np.nonzero(flat == best)[0]
    return np.array(np.unravel_index(winners[0], P.shape)), len(winners) == 1


def grid_edges(H, W):
    """Neighbour pairs of an H x W grid, oriented left-to-right and top-to-bottom,
    with nodes numbered row-major."""
    edges = []
    for r in range(H):
        for c in range(W):
            p = r * W + c
            if c + 1 < W:
                edges.append((p, p + 1))
            if r + 1 < H:
                edges.append((p, p + W))
    return edges


def enumerate_states(n, M):
    """All joint states in lexicographic order (for explicit checks)."""
    return itertools.product(range(M), repeat=n)
