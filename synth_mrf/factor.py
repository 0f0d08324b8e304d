"""Seeded factor-graph workload with higher-order (triple) factors.

Variables on an H x W grid carry the unary of a synthetic slanted-plane
stereo pair (the Sec. 6 stand-in); every three consecutive pixels along a
row or a column share a second-order smoothness factor, compatible where
neighbouring disparities differ by at most T1 and the discrete second
difference is at most T2, with f = exp(-a1 (|x_i - x_j| + |x_j - x_k|) -
a2 |x_i - 2 x_j + x_k|) there and a constant fbar below every compatible
value elsewhere.  Inputs only: no belief-propagation arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .stereo import make_stereo


@dataclass
class FactorGridSpec:
    n_vars: int
    M: int
    factor_vars: np.ndarray   # [n_factors, 3]
    factor_type: np.ndarray   # [n_factors]
    types: list               # [(arity, tuples [C, 3], values float32 [C], fbar)]
    unary: np.ndarray         # [n_vars, M] float32
    truth: np.ndarray         # [n_vars] ground-truth disparity
    H: int
    W: int


def smoothness_triples(M, T1=4, T2=2, a1=0.3, a2=0.6):
    """Compatible (x_i, x_j, x_k), their values and fbar (one factor type)."""
    tuples, vals = [], []
    for xi in range(M):
        for xj in range(max(0, xi - T1), min(M - 1, xi + T1) + 1):
            for xk in range(max(0, xj - T1), min(M - 1, xj + T1) + 1):
                s = abs(xi - 2 * xj + xk)
                if s <= T2:
                    tuples.append((xi, xj, xk))
                    vals.append(math.exp(-a1 * (abs(xi - xj) + abs(xj - xk)) - a2 * s))
    fbar = math.exp(-a1 * 2 * (T1 + 1) - a2 * (T2 + 1))
    return np.array(tuples, dtype=np.int32), np.array(vals, dtype=np.float32), float(np.float32(fbar))


def make_factor_grid(H, W, M, seed=0, beta=0.03, sigma=6.0, T1=4, T2=2):
    g32, D, _, _ = make_stereo(H, W, M, beta, sigma, "slanted", seed)
    tuples, vals, fbar = smoothness_triples(M, T1, T2)
    fv = []
    for r in range(H):
        for c in range(W):
            p = r * W + c
            if c + 2 < W:
                fv.append((p, p + 1, p + 2))
            if r + 2 < H:
                fv.append((p, p + W, p + 2 * W))
    fv = np.array(fv, dtype=np.int32).reshape(-1, 3)
    return FactorGridSpec(H * W, M, fv, np.zeros(len(fv), dtype=np.int32), [(3, tuples, vals, fbar)],
                          g32.reshape(H * W, M), D.reshape(-1), H, W)
