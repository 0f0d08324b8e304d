"""Coarse-to-fine (multi-scale) BP on the grid, FP64, used in tandem with the
O(mM) update (Sec. 2 and Sec. 6 name multi-scale message updating [2] as
exact in the sense that it does not move BP's fixed points).

TEST INFRASTRUCTURE ONLY: never imported by the product path.

Level 0 is the grid; level l+1 groups the 2 x 2 blocks of level l (sizes
ceil(H/2) x ceil(W/2); blocks at an odd edge have fewer children).
- The unary of a block is the product of its children's unaries, divided
  by its maximum over labels (a per-node scale changes no normalised message
  or belief, and keeps the product of many small values representable).
- The pairwise potential is the same at every level.
- The coarsest level starts from uniform messages; every finer level starts
  from its parent's inbox (each child copies the messages into its block),
  then runs its own iterations with the chosen schedule.
"""
from __future__ import annotations

import numpy as np

from . import grid_bp as gb


def coarse_unary(g):
    """[H, W, M] -> [ceil(H/2), ceil(W/2), M]: product over each 2 x 2 block,
    normalised to a maximum of 1 per block."""
    H, W, M = g.shape
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    out = np.ones((Hc, Wc, M))
    for dr in (0, 1):
        for dc in (0, 1):
            part = g[dr::2, dc::2]
            out[: part.shape[0], : part.shape[1]] *= part
    return out / out.max(axis=-1, keepdims=True)


def pyramid(g, levels, storage=None):
    """Unaries of levels 0..levels (level 0 is g itself)."""
    gs = [np.asarray(g, dtype=np.float64)]
    for _ in range(levels):
        gs.append(gb.stored(coarse_unary(gs[-1]), storage))
    return gs


def prolong(coarse_inbox, H, W):
    """Initial inbox of a level from its parent level's inbox: pixel (r, c)
    takes the inbox of block (r // 2, c // 2)."""
    r = np.arange(H) // 2
    c = np.arange(W) // 2
    return coarse_inbox[:, r][:, :, c].copy()


def run(g, pot, mode, levels, iters, schedule=gb.SYNC, impl=gb.SPARSE, storage=None):
    """Multi-scale BP: iters[l] iterations at level l, coarsest (l = levels)
    first.  Returns the level-0 state."""
    assert len(iters) == levels + 1
    gs = pyramid(g, levels, storage)
    state = None
    for lev in range(levels, -1, -1):
        H, W, _ = gs[lev].shape
        init = None if state is None else prolong(state, H, W)
        state = gb.run(gs[lev], pot, mode, iters[lev], schedule, impl, inbox=init, storage=storage)
    return state
