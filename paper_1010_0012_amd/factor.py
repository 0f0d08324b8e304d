"""Convenience wrapper over one bp_fgraph handle (factor graphs with
sparse-compatible higher-order factors).  torch owns the workspace, the
unary and the outputs; every update runs in libbp_hip.so."""
from __future__ import annotations

import torch

from . import _lib as L
from .grid import MODES


class FactorGraph:
    """n_vars variables with M labels; factor a has type factor_type[a] over
    factor_vars[a] (three entries, the third ignored for arity 2); types =
    [(arity, tuples [C, arity], values [C], fbar), ...] on the host.

    >>> fg = FactorGraph(n_vars, M, factor_vars, factor_type, types)
    >>> fg.set_unary(g_cuda); fg.iterate("sum", 20); b = fg.beliefs()
    """

    def __init__(self, n_vars, M, factor_vars, factor_type, types, dense_tables=False, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.n_vars, self.M = n_vars, M
        self.n_factors = len(factor_type)
        with torch.cuda.device(self.device):
            self.handle = L.bp_fg_init(n_vars, M, factor_vars, factor_type, types, dense_tables,
                                       torch.cuda.current_stream(self.device).cuda_stream)
            nbytes = L.bp_fg_workspace_bytes(self.handle)
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws.data_ptr()) % 256
            L.bp_fg_attach_workspace(self.handle, self._ws.data_ptr() + off, nbytes)
        self._g = None

    def _sync_stream(self):
        L.bp_fg_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)

    def set_unary(self, g):
        assert g.is_cuda and g.dtype == torch.float32 and g.is_contiguous()
        assert tuple(g.shape) == (self.n_vars, self.M)
        self._g = g
        L.bp_fg_set_unary(self.handle, g)

    def reset(self):
        self._sync_stream()
        L.bp_fg_reset_messages(self.handle)

    def iterate(self, mode="sum", n_iters=1, dense=False):
        self._sync_stream()
        L.bp_fg_iterate(self.handle, MODES[mode] if isinstance(mode, str) else int(mode), n_iters, dense)

    def beliefs(self):
        out = torch.empty((self.n_vars, self.M), dtype=torch.float32, device=self.device)
        self._sync_stream()
        L.bp_fg_beliefs(self.handle, out, None)
        return out

    def map_labels(self):
        out = torch.empty(self.n_vars, dtype=torch.int32, device=self.device)
        self._sync_stream()
        L.bp_fg_beliefs(self.handle, None, out)
        return out

    def messages(self):
        """(factor->variable, variable->factor), each [n_factors, 3, M]."""
        m = torch.empty((self.n_factors, 3, self.M), dtype=torch.float32, device=self.device)
        n = torch.empty_like(m)
        self._sync_stream()
        L.bp_fg_get_messages(self.handle, m, n)
        return m, n

    def close(self):
        if self.handle:
            L.bp_fg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
