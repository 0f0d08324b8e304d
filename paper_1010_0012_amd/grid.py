"""Convenience wrapper over one bp_grid handle.

torch owns every device buffer (workspace, unary, outputs); the wrapper keeps
references so borrowed pointers stay valid, and enqueues on torch's current
stream of the grid's device.  All compute happens in libbp_hip.so.
"""
from __future__ import annotations

import math

import torch

from . import _lib as L

MODES = {"sum": L.BP_SUM_PRODUCT, "max": L.BP_MAX_PRODUCT}
SCHEDULES = {"sync": L.BP_SCHED_SYNC, "checkerboard": L.BP_SCHED_CHECKERBOARD, "sweep": L.BP_SCHED_SWEEP}


def _as_code(v, table):
    return table[v] if isinstance(v, str) else int(v)


class Grid:
    """An H x W grid MRF with the truncated-linear potential.

    >>> grid = Grid(H, W); grid.set_potential(M, T, alpha)
    >>> grid.set_unary(g_cuda); grid.iterate("sum", 50, "sync")
    >>> b = grid.beliefs(); lab = grid.map_labels()
    """

    def __init__(self, H, W, device=None, stream=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self._stream = stream
            self.handle = L.bp_init_grid(H, W, self._stream_ptr())
        self.H, self.W = H, W
        self.M = None
        self._ws = None
        self._g = None

    def _stream_ptr(self):
        if self._stream is not None:
            return self._stream.cuda_stream
        return torch.cuda.current_stream(self.device).cuda_stream

    def _sync_stream(self):
        L.bp_set_stream(self.handle, self._stream_ptr())

    def set_potential(self, M, T, alpha, fbar=None):
        """fbar=None ties fbar to f(T) = exp(-alpha T) (the library rounds it
        once, so f = exp(-alpha min(|d|, T)) exactly in float32)."""
        tied = fbar is None
        L.bp_set_potential(self.handle, M, T, float(alpha), L.BP_FBAR_TIED if tied else float(fbar))
        self.T, self.alpha = T, float(alpha)
        self.fbar = math.exp(-alpha * T) if tied else float(fbar)
        self.fbar_tied = tied
        if M != self.M:
            self.M = M
            nbytes = L.bp_workspace_bytes(self.handle)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws.data_ptr()) % 256
            self._sync_stream()
            L.bp_attach_workspace(self.handle, self._ws.data_ptr() + off, nbytes)
            self._g = None

    def set_sparse_potentials(self, types, type_h=None, type_v=None):
        """General sparse-compatible potentials: types = [(col_ptr, row_idx,
        val, fbar), ...] host CSR arrays over the second node's label (see
        bp_set_sparse_potentials); type_h [H, W-1] / type_v [H-1, W] uint8
        CUDA tensors or None (type 0).  The tables live in a tensor this
        wrapper keeps; set_potential switches back."""
        assert self.M is not None, "set_potential first (it fixes M)"
        for t, shape in ((type_h, (self.H, self.W - 1)), (type_v, (self.H - 1, self.W))):
            if t is not None:
                assert t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous() and tuple(t.shape) == shape
        nbytes = L.bp_sparse_table_bytes(self.handle, types)
        self._tables = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._tables.data_ptr()) % 256
        self._type_maps = (type_h, type_v)
        self._sync_stream()
        L.bp_set_sparse_potentials(self.handle, types, self._tables.data_ptr() + off, nbytes, type_h, type_v)

    def set_unary(self, g):
        assert g.is_cuda and g.dtype == torch.float32 and g.is_contiguous()
        assert tuple(g.shape) == (self.H, self.W, self.M), (tuple(g.shape), (self.H, self.W, self.M))
        self._g = g
        L.bp_set_unary(self.handle, g)

    def reset(self):
        self._sync_stream()
        L.bp_reset_messages(self.handle)

    def set_sync_fusion(self, enable):
        """Two synchronous iterations per launch (default on; same results)."""
        L.bp_set_sync_fusion(self.handle, enable)

    def set_arithmetic(self, arith):
        """"f64" (default) or "f32": the arithmetic of the sum-product window
        update where a float32 kernel is compiled (bp_set_arithmetic)."""
        L.bp_set_arithmetic(self.handle, {"f64": L.BP_ARITH_F64, "f32": L.BP_ARITH_F32}[arith])

    def message_stats(self):
        """(largest |m - m'| against the other message buffer, number of
        non-finite entries) of the current messages (bp_message_stats);
        waits for the stream."""
        self._sync_stream()
        out = torch.empty(2, dtype=torch.int32, device=self.device)
        L.bp_message_stats(self.handle, out.data_ptr(), out.data_ptr() + 4)
        torch.cuda.synchronize(self.device)
        v = out.cpu()
        return float(v[:1].view(torch.float32)[0]), int(v[1])

    LAYOUTS = {"strips": 0, "bands": 1, "slots": 2, "wide": 3, "walk": 4, "tile": 5}

    def set_launch_tuning(self, layout="wide", cap=-1):
        """Mapping of the two-iteration launches ("strips", "wide", "bands" or "slots")
        and their workgroups per CU (0 none, -1 the default); every setting
        gives the same bits (bp_set_launch_tuning)."""
        L.bp_set_launch_tuning(self.handle, self.LAYOUTS[layout], cap)

    def get_launch_tuning(self):
        layout, cap = L.bp_get_launch_tuning(self.handle)
        return {v: k for k, v in self.LAYOUTS.items()}[layout], cap

    def autotune(self, mode="sum", schedule="sync", trial_iters=4):
        """Time the launch mappings on this grid and keep the fastest
        (bp_autotune); resets the messages.  Returns us per iteration."""
        self._sync_stream()
        return L.bp_autotune(self.handle, MODES[mode] if isinstance(mode, str) else int(mode),
                             SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule), trial_iters)

    def iterate(self, mode="sum", n_iters=1, schedule="sync", dense=False):
        self._sync_stream()
        fn = L.bp_iterate_dense if dense else L.bp_iterate
        fn(self.handle, _as_code(mode, MODES), n_iters, _as_code(schedule, SCHEDULES))

    def iterate_multiscale(self, mode="sum", iters=(10, 10, 10)):
        """Coarse-to-fine solve: iters[l] synchronous iterations at level l
        (iters[0] the finest), len(iters) - 1 coarser levels."""
        levels = len(iters) - 1
        nbytes = L.bp_multiscale_workspace_bytes(self.handle, levels)
        if getattr(self, "_ms_ws", None) is None or self._ms_ws.numel() < nbytes + 256:
            self._ms_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ms_ws.data_ptr()) % 256
        self._sync_stream()
        L.bp_iterate_multiscale(self.handle, _as_code(mode, MODES), list(iters), self._ms_ws.data_ptr() + off, nbytes)

    def beliefs(self, out=None):
        if out is None:
            out = torch.empty((self.H, self.W, self.M), dtype=torch.float32, device=self.device)
        self._sync_stream()
        L.bp_beliefs(self.handle, out)
        return out

    def map_labels(self, out=None):
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device)
        self._sync_stream()
        L.bp_map_labels(self.handle, out)
        return out

    def readout(self, beliefs=None, labels=None):
        """Beliefs and MAP labels in one pass over the messages."""
        if beliefs is None:
            beliefs = torch.empty((self.H, self.W, self.M), dtype=torch.float32, device=self.device)
        if labels is None:
            labels = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device)
        self._sync_stream()
        L.bp_readout(self.handle, beliefs, labels)
        return beliefs, labels

    def get_messages(self, out=None):
        if out is None:
            out = torch.empty((4, self.H, self.W, self.M), dtype=torch.float32, device=self.device)
        self._sync_stream()
        L.bp_get_messages(self.handle, out)
        return out

    def set_messages(self, src):
        assert src.is_cuda and src.dtype == torch.float32 and src.is_contiguous()
        assert tuple(src.shape) == (4, self.H, self.W, self.M)
        self._sync_stream()
        L.bp_set_messages(self.handle, src)

    def close(self):
        if self.handle:
            L.bp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
