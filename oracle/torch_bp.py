"""Differentiable forward of synchronous sum-product grid BP in plain PyTorch (CPU, FP64).

TEST INFRASTRUCTURE ONLY: never imported by the product path.

Written independently of grid_bp/grad_ref (outbox layout, padding with ones
for missing neighbours, dense Eq. 2 products) so that autograd through it is
a check on the hand-written adjoint rather than a copy of it.
"""
from __future__ import annotations

import torch


def _potential(M, T, alpha, fbar=None):
    x = torch.arange(M, dtype=torch.float64)
    d = (x[:, None] - x[None, :]).abs()
    fb = torch.exp(-alpha * T) if fbar is None else torch.as_tensor(fbar, dtype=torch.float64)
    return torch.where(d <= T, torch.exp(-alpha * d), fb * torch.ones_like(d))


def _incoming(out_r, out_l, out_d, out_u):
    """Messages arriving at every pixel from its left/right/up/down neighbour,
    padded with ones where the neighbour is missing.  out_X[p] is the message
    pixel p sends towards direction X."""
    H, W, M = out_r.shape
    one_col = torch.ones(H, 1, M, dtype=out_r.dtype)
    one_row = torch.ones(1, W, M, dtype=out_r.dtype)
    from_left = torch.cat([one_col, out_r[:, :-1]], dim=1)
    from_right = torch.cat([out_l[:, 1:], one_col], dim=1)
    from_up = torch.cat([one_row, out_d[:-1]], dim=0)
    from_down = torch.cat([out_u[1:], one_row], dim=0)
    return from_left, from_right, from_up, from_down


def forward(theta, alpha, T, n_iters, fbar=None):
    """Beliefs after n sync iterations from uniform messages; theta = log g."""
    H, W, M = theta.shape
    g = torch.exp(theta)
    F = _potential(M, T, alpha, fbar)
    u0 = torch.full((H, W, M), 1.0 / M, dtype=torch.float64)
    out_r = out_l = out_d = out_u = u0
    for _ in range(n_iters):
        fl, fr, fu, fd = _incoming(out_r, out_l, out_d, out_u)
        # sending right: exclude what came from the right, and so on
        h_r = g * fl * fu * fd
        h_l = g * fr * fu * fd
        h_d = g * fl * fr * fu
        h_u = g * fl * fr * fd
        # a rightward/downward message uses F[x_sender, x_receiver]; leftward/upward F^T
        new = []
        for h, K in ((h_r, F), (h_l, F.T), (h_d, F), (h_u, F.T)):
            u = h @ K
            new.append(u / u.sum(dim=-1, keepdim=True))
        out_r, out_l, out_d, out_u = new
    fl, fr, fu, fd = _incoming(out_r, out_l, out_d, out_u)
    b = g * fl * fr * fu * fd
    return b / b.sum(dim=-1, keepdim=True)


def ce_loss(b, labels):
    idx = torch.as_tensor(labels, dtype=torch.long)[..., None]
    return -torch.log(torch.gather(b, -1, idx)).mean()


def autograd_grad(g, labels, T, alpha, n_iters, fbar=None):
    """(loss, dL/dtheta, dL/dalpha) by torch.autograd in FP64."""
    theta = torch.log(torch.as_tensor(g, dtype=torch.float64)).requires_grad_(True)
    a = torch.tensor(float(alpha), dtype=torch.float64, requires_grad=True)
    L = ce_loss(forward(theta, a, T, n_iters, fbar), labels)
    L.backward()
    return float(L.detach()), theta.grad.numpy(), float(a.grad)
