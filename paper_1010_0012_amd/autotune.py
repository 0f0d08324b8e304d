"""Plan cache for the batched path.

bp_batch_autotune (in the library) times candidate work plans on the device
and keeps the fastest; this module remembers the winner per batch signature
(the (H, W, M, T) of every instance) in a JSON file so later runs reuse it
with bp_batch_set_streams / bp_batch_set_plan instead of searching again.
"""
from __future__ import annotations

import hashlib
import json
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bp_batch_plans.json")


def signature_key(batch, mode):
    raw = json.dumps({"mode": mode, "grids": batch.signature()}, sort_keys=True)
    return hashlib.sha256(raw.encode()).hexdigest()[:32]


def tuned_plan(batch, mode="sum", trial_iters=3, cache_path=DEFAULT_CACHE):
    """Apply the cached plan for this batch, or autotune and cache it.
    Returns (passes, grid_blocks, streams, best_us or None when taken from
    the cache)."""
    key = signature_key(batch, mode)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if key in cache and "streams" in cache[key]:
        passes, grid, streams = cache[key]["passes"], cache[key]["grid_blocks"], cache[key]["streams"]
        batch.set_streams(streams)
        batch.set_plan(passes, grid)
        return passes, grid, streams, None
    best_us = batch.autotune(mode, trial_iters)
    passes, grid = batch.get_plan()
    streams = batch.get_streams()
    if cache_path:
        cache[key] = {"passes": passes, "grid_blocks": grid, "streams": streams, "best_us": best_us}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return passes, grid, streams, best_us
