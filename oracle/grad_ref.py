"""FP64 adjoint of unrolled synchronous sum-product BP on the grid.

TEST INFRASTRUCTURE ONLY: never imported by the product path.

Sum-product beliefs are differentiable functions of the unary and of the
potential's parameters, which is what marginal-based parameter learning needs
(Sec. 1 and Sec. 7 motivate sum-product BP for maximum-likelihood / CRF
estimation).  This module differentiates

    L = -(1/N) * sum_p log b_p(y_p)          (mean cross-entropy vs labels y)

through n synchronous iterations started from uniform messages, with respect
to theta = log g (per pixel and label) and the smoothness weight alpha of the
truncated-linear potential f(d) = exp(-alpha |d|), |d| <= T, with fbar either
tied to alpha (fbar = exp(-alpha T), the Sec. 1 form) or held fixed.

Reverse step (derived from the forward recursion, written out here):
for a message e = p -> q with h_e from Eq. 5, u_e = F-product of h_e (Eq. 2),
Z_e = sum u_e and m_e = u_e / Z_e, and lambda_e = dL/dlog m_e:

    mu     = lambda_e - m_e * sum(lambda_e)
    ubar   = mu / u_e                       (dL/du_e)
    hbar   = F applied to ubar from the other side (transposed product)
    eta    = hbar * h_e                     (dL/dlog h_e)
    theta_bar_p          += eta
    lambda^t_{k -> p}    += eta   for every neighbour k of p except q
    alpha_bar            += sum_{x,y} dF(x,y)/dalpha * h_e(x) * ubar(y)

Seed from the loss: dL/d(log-belief logits at p) = (b_p - onehot(y_p)) / N,
which feeds theta_bar_p directly and lambda^n on every message into p.
"""
from __future__ import annotations

import numpy as np

from . import grid_bp as gb


def potential_and_derivative(M, T, alpha, fbar=None):
    """Truncated-linear potential and dF/dalpha.

    fbar=None ties fbar = exp(-alpha T) (so its derivative is -T fbar);
    a given fbar is a constant (derivative 0).
    """
    pot = gb.truncated_linear(M, T, alpha, fbar)
    x = np.arange(M)
    d = np.abs(x[:, None] - x[None, :]).astype(np.float64)
    dfbar = -T * pot.fbar if fbar is None else 0.0
    dF = np.where(pot.compat, -d * np.exp(-alpha * d), dfbar)
    return pot, dF


def forward_states(g, pot, n_iters):
    """All sync states m^0 .. m^n of sum-product BP (dense form, Eq. 2)."""
    _, states = gb.run(g, pot, gb.SUM, n_iters, gb.SYNC, gb.DENSE, record=True)
    return states


def loss(g, inbox, labels):
    b = gb.beliefs(g, inbox)
    H, W, _ = b.shape
    r, c = np.mgrid[0:H, 0:W]
    return -np.mean(np.log(b[r, c, labels])), b


def loss_of(g, labels, M, T, alpha, n_iters, fbar=None):
    """Forward only: the scalar loss (for finite differences)."""
    pot = gb.truncated_linear(M, T, alpha, fbar)
    state = gb.run(np.asarray(g, np.float64), pot, gb.SUM, n_iters, gb.SYNC, gb.DENSE)
    return loss(g, state, labels)[0]


def seed_from_beliefs(b, labels):
    """dL/d(logits) of the mean cross-entropy: (b - onehot(y)) / N."""
    H, W, M = b.shape
    onehot = np.zeros_like(b)
    r, c = np.mgrid[0:H, 0:W]
    onehot[r, c, labels] = 1.0
    return (b - onehot) / (H * W)


def seed_from_belief_grad(b, dL_db):
    """dL/d(logits) for a general loss with gradient dL_db on normalised beliefs."""
    return b * (dL_db - np.sum(b * dL_db, axis=-1, keepdims=True))


def reverse_step(g, m_t, lam_next, pot, dF):
    """One reverse synchronous step.

    m_t      : state at time t (inputs of the step), [4, H, W, M]
    lam_next : dL/dlog m^{t+1}, in inbox layout, [4, H, W, M]
    Returns (lam_t, theta_bar_increment, alpha_bar_increment).
    """
    H, W, M = g.shape
    has = gb.has_neighbor(H, W)
    lam_t = np.zeros_like(m_t)
    theta_inc = np.zeros((H, W, M))
    alpha_inc = 0.0
    for o in gb.DIRS:
        dr, dc = gb.OFFSETS[o]
        (rs, rq), (cs, cq) = gb._span(dr, H), gb._span(dc, W)
        P = gb.oriented_potential(pot, o).F            # P[x_sender, x_receiver]
        dP = dF if o in (gb.RIGHT, gb.DOWN) else dF.T
        h = gb.h_vector(g, m_t, has, o)[rs, cs]         # senders only
        u = h @ P
        m_new = u / u.sum(axis=-1, keepdims=True)
        lam_e = lam_next[gb.OPPOSITE[o], rq, cq]         # dL/dlog m_{p->q}
        mu = lam_e - m_new * lam_e.sum(axis=-1, keepdims=True)
        ubar = mu / u
        hbar = ubar @ P.T
        eta = hbar * h
        theta_inc[rs, cs] += eta
        for k in gb.DIRS:
            if k == o:
                continue
            sel = has[k, rs, cs]
            blk = lam_t[k, rs, cs]
            blk[sel] += eta[sel]
            lam_t[k, rs, cs] = blk
        alpha_inc += float(np.sum(h * (ubar @ dP.T)))
    return lam_t, theta_inc, alpha_inc


def grad(g, labels, M, T, alpha, n_iters, fbar=None, dL_db=None):
    """Loss, dL/dtheta ([H, W, M]) and dL/dalpha for n synchronous iterations.

    With dL_db given, the loss is the caller's (its gradient on beliefs) and
    the returned loss value is None.
    """
    g = np.asarray(g, dtype=np.float64)
    H, W, _ = g.shape
    pot, dF = potential_and_derivative(M, T, alpha, fbar)
    states = forward_states(g, pot, n_iters)
    L, b = loss(g, states[-1], labels) if labels is not None else (None, gb.beliefs(g, states[-1]))
    a_bar = seed_from_beliefs(b, labels) if dL_db is None else seed_from_belief_grad(b, dL_db)
    has = gb.has_neighbor(H, W)
    theta_bar = a_bar.copy()
    lam = np.where(has[..., None], a_bar[None], 0.0)
    alpha_bar = 0.0
    for t in range(n_iters - 1, -1, -1):
        lam, th, al = reverse_step(g, states[t], lam, pot, dF)
        theta_bar += th
        alpha_bar += al
    return L, theta_bar, alpha_bar
