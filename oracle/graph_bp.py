"""Plain dense BP on an arbitrary undirected pairwise MRF (edge list), FP64.

TEST INFRASTRUCTURE ONLY: never imported by the product path.

A second, independent implementation of Eq. 2, Eq. 3 and Eq. 9 written per
directed edge with explicit loops over the neighbour lists.  On trees it is
checked against brute force; on grids it cross-checks the vectorised grid
oracle's indexing.
"""
from __future__ import annotations

import numpy as np


class PairwiseMRF:
    def __init__(self, n, M, edges, F_list, g):
        self.n, self.M = n, M
        self.edges = list(edges)
        self.F = [np.asarray(F, dtype=np.float64) for F in F_list]
        self.g = np.asarray(g, dtype=np.float64)
        self.nbrs = [[] for _ in range(n)]
        for e, (a, b) in enumerate(self.edges):
            self.nbrs[a].append((b, e))
            self.nbrs[b].append((a, e))

    def factor(self, i, j, e):
        """Matrix K with K[x_i, x_j] = f(x_i, x_j) for the pair (i, j)."""
        a, _ = self.edges[e]
        return self.F[e] if a == i else self.F[e].T


def run_bp(mrf, mode="sum", n_iters=10):
    """Synchronous BP from uniform messages; returns {(i, j): m_ij} after n_iters."""
    M = mrf.M
    msgs = {}
    for i in range(mrf.n):
        for j, _ in mrf.nbrs[i]:
            msgs[(i, j)] = np.full(M, 1.0 / M)
    for _ in range(n_iters):
        new = {}
        for i in range(mrf.n):
            for j, e in mrf.nbrs[i]:
                h = mrf.g[i].copy()                    # Eq. 5
                for k, _ in mrf.nbrs[i]:
                    if k != j:
                        h = h * msgs[(k, i)]
                K = mrf.factor(i, j, e)
                u = np.zeros(M)
                for xj in range(M):                    # Eq. 2 / Eq. 9, every (x_i, x_j)
                    terms = [K[xi, xj] * h[xi] for xi in range(M)]
                    u[xj] = sum(terms) if mode == "sum" else max(terms)
                new[(i, j)] = u / u.sum()
        msgs = new
    return msgs


def beliefs(mrf, msgs):
    """Eq. 3 per node, [n, M]."""
    out = np.empty((mrf.n, mrf.M))
    for i in range(mrf.n):
        b = mrf.g[i].copy()
        for k, _ in mrf.nbrs[i]:
            b = b * msgs[(k, i)]
        out[i] = b / b.sum()
    return out
