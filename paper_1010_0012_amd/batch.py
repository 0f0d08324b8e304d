"""Convenience wrapper over a bp_batch handle (many independent grid MRFs).

torch owns the unaries, the workspace and the outputs; the wrapper keeps
them alive and splits the concatenated outputs per instance.
"""
from __future__ import annotations

import math

import torch

from . import _lib as L
from .grid import MODES


class Batch:
    """grids: list of (unary [H, W, M] float32 CUDA tensor, T, alpha[, fbar])."""

    def __init__(self, grids, device=None, stream=None, graphs=True):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._stream = stream
        self._g = []
        descs = []
        for spec in grids:
            g, T, alpha = spec[0], spec[1], spec[2]
            fbar = spec[3] if len(spec) > 3 else None
            assert g.is_cuda and g.dtype == torch.float32 and g.is_contiguous() and g.dim() == 3
            H, W, M = g.shape
            self._g.append(g)
            descs.append(L.bp_grid_desc(H, W, M, T, float(alpha),
                                        L.BP_FBAR_TIED if fbar is None else float(fbar), g.data_ptr()))
        self.shapes = [tuple(g.shape) for g in self._g]
        self.params = [(int(s[1]), float(s[2])) for s in grids]
        with torch.cuda.device(self.device):
            self.handle = L.bp_batch_init(descs, self._stream_ptr())
            nbytes = L.bp_batch_workspace_bytes(self.handle)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws.data_ptr()) % 256
            L.bp_batch_attach_workspace(self.handle, self._ws.data_ptr() + off, nbytes)
        L.bp_batch_set_graphs(self.handle, graphs)
        self.n_beliefs = sum(H * W * M for H, W, M in self.shapes)
        self.n_labels = sum(H * W for H, W, _ in self.shapes)

    def _stream_ptr(self):
        if self._stream is not None:
            return self._stream.cuda_stream
        return torch.cuda.current_stream(self.device).cuda_stream

    def _sync_stream(self):
        L.bp_batch_set_stream(self.handle, self._stream_ptr())

    def signature(self):
        """Shape key for plan caching: (H, W, M, T) of every instance."""
        return [[H, W, M, T] for (H, W, M), (T, _) in zip(self.shapes, self.params)]

    def reset(self):
        self._sync_stream()
        L.bp_batch_reset_messages(self.handle)

    def iterate(self, mode="sum", n_iters=1):
        self._sync_stream()
        L.bp_batch_iterate(self.handle, MODES[mode] if isinstance(mode, str) else int(mode), n_iters)

    def set_arithmetic(self, arith):
        """"f64" (default) or "f32": the arithmetic of the sum-product updates
        of the instances that have a float32 kernel (bp_batch_set_arithmetic)."""
        L.bp_batch_set_arithmetic(self.handle, {"f64": L.BP_ARITH_F64, "f32": L.BP_ARITH_F32}[arith])

    def set_plan(self, passes, grid_blocks):
        self._sync_stream()
        L.bp_batch_set_plan(self.handle, passes, grid_blocks)

    def get_plan(self):
        return L.bp_batch_get_plan(self.handle)

    def set_streams(self, n_streams):
        self._sync_stream()
        L.bp_batch_set_streams(self.handle, n_streams)

    def get_streams(self):
        return L.bp_batch_get_streams(self.handle)

    def autotune(self, mode="sum", trial_iters=3):
        self._sync_stream()
        return L.bp_batch_autotune(self.handle, MODES[mode] if isinstance(mode, str) else int(mode),
                                   trial_iters)

    def beliefs(self, split=True):
        out = torch.empty(self.n_beliefs, dtype=torch.float32, device=self.device)
        self._sync_stream()
        L.bp_batch_beliefs(self.handle, out)
        return self._split(out, [H * W * M for H, W, M in self.shapes],
                           [(H, W, M) for H, W, M in self.shapes]) if split else out

    def map_labels(self, split=True):
        out = torch.empty(self.n_labels, dtype=torch.int32, device=self.device)
        self._sync_stream()
        L.bp_batch_map_labels(self.handle, out)
        return self._split(out, [H * W for H, W, _ in self.shapes],
                           [(H, W) for H, W, _ in self.shapes]) if split else out

    @staticmethod
    def _split(flat, sizes, shapes):
        parts, off = [], 0
        for n, shp in zip(sizes, shapes):
            parts.append(flat[off:off + n].view(shp))
            off += n
        return parts

    def close(self):
        if getattr(self, "handle", None):
            L.bp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fbar_of(T, alpha):
    return math.exp(-alpha * T)
