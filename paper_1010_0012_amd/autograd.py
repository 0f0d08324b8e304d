"""Differentiable sum-product BP: a torch.autograd.Function over the C ABI.

forward(theta, alpha): g = exp(theta) is handed to the library as the unary,
n synchronous sum-product iterations run with message checkpoints every k
(bp_forward_ckpt), and the beliefs of the final state are returned.
backward(dL/db): bp_backward runs the hand-written adjoint kernels and
returns dL/dtheta and dL/dalpha.  Both passes run in libbp_hip.so; the only
torch compute is the exp that maps the caller's log-unary to g.

A grid handle keeps the checkpoints of its latest forward only.  Each
forward is stamped with a per-grid generation; a backward whose forward is
no longer the grid's latest (another forward on the same grid, or any call
that changed its state) first replays its own forward into its own
workspace, which is deterministic and so restores the same checkpoints bit
for bit.
"""
from __future__ import annotations

import itertools

import torch

from . import _lib as L
from .grid import Grid

_generation = itertools.count(1)


def _forward(grid, g, alpha, T, fbar, n_iters, ckpt_every, gws, off, nbytes):
    H, W, M = g.shape
    grid.set_potential(M, T, alpha, fbar)
    grid.set_unary(g)
    grid._sync_stream()
    L.bp_forward_ckpt(grid.handle, n_iters, ckpt_every, gws.data_ptr() + off, nbytes)
    grid._bp_grad_gen = next(_generation)
    return grid._bp_grad_gen


class BPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, alpha, grid, T, n_iters, ckpt_every, fbar=None):
        H, W, M = theta.shape
        g = torch.exp(theta.detach()).contiguous()
        grid.set_potential(M, T, float(alpha), fbar)
        nbytes = L.bp_grad_workspace_bytes(grid.handle, n_iters, ckpt_every)
        gws = torch.empty(nbytes + 256, dtype=torch.uint8, device=theta.device)
        off = (-gws.data_ptr()) % 256
        args = (grid, g, float(alpha), T, fbar, n_iters, ckpt_every, gws, off, nbytes)
        ctx.gen = _forward(*args)
        b = grid.beliefs()
        ctx.args = args
        return b

    @staticmethod
    def backward(ctx, grad_b):
        grid, g = ctx.args[0], ctx.args[1]
        if getattr(grid, "_bp_grad_gen", None) != ctx.gen:
            ctx.gen = _forward(*ctx.args)        # this forward's checkpoints, replayed
        dtheta = torch.empty_like(g)
        dalpha = torch.zeros(1, dtype=torch.float32, device=g.device)
        grid._sync_stream()
        try:
            L.bp_backward(grid.handle, grad_b.contiguous(), dtheta, dalpha)
        except L.BPError as e:
            if e.status != L.BP_ESTATE:
                raise
            # the grid's state changed since this forward (not through a
            # forward of this class): replay it and run the reverse pass
            ctx.gen = _forward(*ctx.args)
            grid._sync_stream()
            L.bp_backward(grid.handle, grad_b.contiguous(), dtheta, dalpha)
        return dtheta, dalpha[0], None, None, None, None, None


def bp_beliefs(theta, alpha, grid: Grid, T, n_iters, ckpt_every=5, fbar=None):
    """Beliefs after n_iters synchronous sum-product iterations, differentiable
    w.r.t. theta (= log g, [H, W, M]) and alpha.  fbar=None ties fbar to
    exp(-alpha T); fbar = 0 is refused (the adjoint needs positive messages)."""
    if not torch.is_tensor(alpha):
        alpha = torch.tensor(float(alpha), device=theta.device)
    return BPFunction.apply(theta, alpha, grid, T, n_iters, ckpt_every, fbar)
