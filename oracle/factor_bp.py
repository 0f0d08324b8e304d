"""FP64 factor-graph BP with sparse-compatible higher-order factors (Sec. 7).

TEST INFRASTRUCTURE ONLY: never imported by the product path.

A factor of arity K (2 or 3) has a table f(x_1, .., x_K) that equals a
constant fbar except on a set C of compatible tuples.  Standard factor BP
(sum-product; max-product in the product domain):
  variable -> factor  n_{v->a}(x) = g_v(x) * prod over the other factors b
                                    of v of m_{b->v}(x), normalised;
  factor -> variable  m_{a->v_i}(x) = sum (max) over the tuples with
                                    x_i = x of f(tuple) * prod_{j != i}
                                    n_{v_j->a}(x_j), normalised.
The dense form visits all M^(K-1) completions per label (O(M^K) per
message).  Splitting the table into fbar plus the compatible part (the
factor analogue of Eq. 6 / Eq. 7) gives
  sum: fbar * prod_{j != i} S_j + sum over C with t_i = x of
       (f(t) - fbar) * prod_{j != i} n_j(t_j),        S_j = sum_x n_j(x);
  max: max(fbar * prod_{j != i} H_j, max over C with t_i = x of
       f(t) * prod_{j != i} n_j(t_j)),                 H_j = max_x n_j(x),
O(C + M) per message; the max form needs f >= fbar on C (as Eq. 11).
Without that condition the split form (the factor analogue of Eq. 6 /
Eq. 10) is exact for max-product:
  max: max(max over C with t_i = x of f(t) * prod_{j != i} n_j(t_j),
           fbar * max over the completions with t_i = x outside C of
           prod_{j != i} n_j(t_j)),
written here by enumerating the completions outside C.
Schedule: synchronous, every variable->factor message from the current
factor->variable messages, then every factor->variable message.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .grid_bp import normalize, stored

SUM, MAX = "sum", "max"
DENSE, SPARSE, SPLIT = "dense", "sparse", "split"


@dataclass
class FactorType:
    """A sparse-compatible factor: tuples [C, K] of labels, values [C], fbar."""

    arity: int
    tuples: np.ndarray
    values: np.ndarray
    fbar: float

    def __post_init__(self):
        self.tuples = np.asarray(self.tuples, dtype=np.int64).reshape(-1, self.arity)
        self.values = np.asarray(self.values, dtype=np.float64)
        assert len(self.tuples) == len(self.values)
        assert len({tuple(t) for t in self.tuples}) == len(self.tuples), "duplicate tuple"

    def table(self, M):
        """The full table f[x_1, .., x_K] (fbar outside C)."""
        F = np.full((M,) * self.arity, float(self.fbar))
        for t, v in zip(self.tuples, self.values):
            F[tuple(t)] = v
        return F


@dataclass
class FactorGraph:
    """n_vars variables with M labels; factors[a] = (variables, type index)."""

    n_vars: int
    M: int
    factors: list
    types: list

    def __post_init__(self):
        self.adj = [[] for _ in range(self.n_vars)]   # (factor, slot) per variable, in factor order
        for a, (vs, k) in enumerate(self.factors):
            assert len(vs) == self.types[k].arity and len(set(vs)) == len(vs)
            for i, v in enumerate(vs):
                self.adj[v].append((a, i))


def init_messages(fg):
    """Uniform factor->variable messages m[a][i] (and variable->factor n)."""
    return [[np.full(fg.M, 1.0 / fg.M) for _ in vs] for vs, _ in fg.factors]


def var_to_factor(fg, g, m, storage=None):
    """n[a][i]: g_v times the messages of v's other factors (adjacency order)."""
    n = [[None] * len(vs) for vs, _ in fg.factors]
    for v in range(fg.n_vars):
        for a, i in fg.adj[v]:
            p = np.array(g[v], dtype=np.float64)
            for b, j in fg.adj[v]:
                if (b, j) != (a, i):
                    p = p * m[b][j]
            n[a][i] = stored(normalize(p), storage)
    return n


def factor_message_dense(fg, a, i, n, mode):
    """Every completion of the other slots, O(M^K)."""
    vs, k = fg.factors[a]
    F = fg.types[k].table(fg.M)
    prod = F
    for j in range(len(vs)):
        if j == i:
            continue
        shape = [1] * len(vs)
        shape[j] = fg.M
        prod = prod * n[a][j].reshape(shape)
    axes = tuple(j for j in range(len(vs)) if j != i)
    return prod.sum(axis=axes) if mode == SUM else prod.max(axis=axes)


def factor_message_sparse(fg, a, i, n, mode):
    """fbar term once per message plus the compatible tuples, O(C + M)."""
    vs, k = fg.factors[a]
    ft = fg.types[k]
    others = [j for j in range(len(vs)) if j != i]

    def chain(first, factors):
        # products left to right, the order of the dense form
        p = first
        for x in factors:
            p = p * x
        return p

    if mode == SUM:
        base = chain(ft.fbar, [n[a][j].sum() for j in others])
        u = np.full(fg.M, base)
        for t, f in zip(ft.tuples, ft.values):
            u[t[i]] += chain(f - ft.fbar, [n[a][j][t[j]] for j in others])
    else:
        base = chain(ft.fbar, [n[a][j].max() for j in others])
        u = np.full(fg.M, base)
        for t, f in zip(ft.tuples, ft.values):
            u[t[i]] = max(u[t[i]], chain(f, [n[a][j][t[j]] for j in others]))
    return u


def factor_message_split(fg, a, i, n, mode):
    """Max-product: the compatible tuples with their own f, and fbar times the
    largest product over the completions outside C (enumerated), each
    product taken left to right as in the dense form.  Sum-product is the
    sparse form (Eq. 7's analogue is exact for any fbar)."""
    if mode == SUM:
        return factor_message_sparse(fg, a, i, n, mode)
    vs, k = fg.factors[a]
    ft = fg.types[k]
    others = [j for j in range(len(vs)) if j != i]
    listed = {tuple(t) for t in ft.tuples}
    u = np.zeros(fg.M)
    for t, f in zip(ft.tuples, ft.values):
        p = f
        for j in others:
            p = p * n[a][j][t[j]]
        u[t[i]] = max(u[t[i]], p)
    for t in itertools.product(range(fg.M), repeat=len(vs)):
        if t in listed:
            continue
        p = ft.fbar
        for j in others:
            p = p * n[a][j][t[j]]
        u[t[i]] = max(u[t[i]], p)
    return u


def factor_to_var(fg, n, mode, impl, storage=None):
    form = {DENSE: factor_message_dense, SPARSE: factor_message_sparse, SPLIT: factor_message_split}[impl]
    return [[stored(normalize(form(fg, a, i, n, mode)), storage) for i in range(len(vs))]
            for a, (vs, _) in enumerate(fg.factors)]


def run(fg, g, mode=SUM, n_iters=10, impl=SPARSE, storage=None):
    """Synchronous factor BP from uniform messages; returns (m, n)."""
    g = np.asarray(g, dtype=np.float64)
    m = [[stored(x, storage) for x in row] for row in init_messages(fg)]
    n = m
    for _ in range(n_iters):
        n = var_to_factor(fg, g, m, storage)
        m = factor_to_var(fg, n, mode, impl, storage)
    return m, n


def beliefs(fg, g, m):
    """b_v proportional to g_v times every incoming factor message."""
    out = np.empty((fg.n_vars, fg.M))
    for v in range(fg.n_vars):
        b = np.array(g[v], dtype=np.float64)
        for a, i in fg.adj[v]:
            b = b * m[a][i]
        out[v] = b / b.sum()
    return out


def brute_marginals(fg, g, mode=SUM):
    """Exact (max-)marginals by enumerating all M^n states (tiny graphs)."""
    M, nv = fg.M, fg.n_vars
    out = np.zeros((nv, M))
    tables = [fg.types[k].table(M) for _, k in fg.factors]
    for x in itertools.product(range(M), repeat=nv):
        p = 1.0
        for v in range(nv):
            p *= g[v][x[v]]
        for (vs, _), F in zip(fg.factors, tables):
            p *= F[tuple(x[v] for v in vs)]
        for v in range(nv):
            out[v, x[v]] = out[v, x[v]] + p if mode == SUM else max(out[v, x[v]], p)
    return out / out.sum(axis=1, keepdims=True)
