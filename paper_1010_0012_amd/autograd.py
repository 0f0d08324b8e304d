"""Differentiable sum-product BP: a torch.autograd.Function over the C ABI.

forward(theta, alpha): g = exp(theta) is handed to the library as the unary,
n synchronous sum-product iterations run with message checkpoints every k
(bp_forward_ckpt), and the beliefs of the final state are returned.
backward(dL/db): bp_backward runs the hand-written adjoint kernels and
returns dL/dtheta and dL/dalpha.  Both passes run in libbp_hip.so; the only
torch compute is the exp that maps the caller's log-unary to g.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .grid import Grid


class BPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, alpha, grid, T, n_iters, ckpt_every, fbar=None):
        H, W, M = theta.shape
        g = torch.exp(theta.detach()).contiguous()
        grid.set_potential(M, T, float(alpha), fbar)
        grid.set_unary(g)
        nbytes = L.bp_grad_workspace_bytes(grid.handle, n_iters, ckpt_every)
        gws = torch.empty(nbytes + 256, dtype=torch.uint8, device=theta.device)
        off = (-gws.data_ptr()) % 256
        grid._sync_stream()
        L.bp_forward_ckpt(grid.handle, n_iters, ckpt_every, gws.data_ptr() + off, nbytes)
        b = grid.beliefs()
        ctx.grid, ctx.g, ctx.gws = grid, g, gws
        return b

    @staticmethod
    def backward(ctx, grad_b):
        grid = ctx.grid
        dtheta = torch.empty_like(ctx.g)
        dalpha = torch.zeros(1, dtype=torch.float32, device=ctx.g.device)
        grid._sync_stream()
        L.bp_backward(grid.handle, grad_b.contiguous(), dtheta, dalpha)
        return dtheta, dalpha[0], None, None, None, None, None


def bp_beliefs(theta, alpha, grid: Grid, T, n_iters, ckpt_every=5, fbar=None):
    """Beliefs after n_iters synchronous sum-product iterations, differentiable
    w.r.t. theta (= log g, [H, W, M]) and alpha.  fbar=None ties fbar to
    exp(-alpha T)."""
    if not torch.is_tensor(alpha):
        alpha = torch.tensor(float(alpha), device=theta.device)
    return BPFunction.apply(theta, alpha, grid, T, n_iters, ckpt_every, fbar)
