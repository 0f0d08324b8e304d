"""ctypes binding of libbp_hip.so: one Python function per C entry point,
same names, argument marshalling only.

Device buffers are passed as torch CUDA tensors (or raw integer device
addresses); the HIP stream defaults to torch's current stream on the handle's
device.  Every status < 0 raises BPError with the library's message.  There is
no CPU fallback: if the shared library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libbp_hip.so")
HEADER = os.path.join(os.path.dirname(PKG_DIR), "include", "bp.h")

BP_OK, BP_EINVAL, BP_ESTATE, BP_ENOMEM, BP_EHIP, BP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BP_SUM_PRODUCT, BP_MAX_PRODUCT = 0, 1
BP_SCHED_SYNC, BP_SCHED_CHECKERBOARD, BP_SCHED_SWEEP = 0, 1, 2
BP_MAX_LABELS = 256
BP_FBAR_TIED = -1.0
BP_ARITH_F64, BP_ARITH_F32 = 0, 1
BP_PAIR_STRIPS, BP_PAIR_BANDS, BP_PAIR_SLOTS, BP_PAIR_WIDE, BP_PAIR_WALK, BP_PAIR_TILE = 0, 1, 2, 3, 4, 5

_c_int, _c_i32, _c_i64, _c_f, _vp = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p


class bp_grid_desc(ctypes.Structure):
    """struct bp_grid_desc (include/bp.h)."""
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("M", ctypes.c_int32),
                ("T", ctypes.c_int32), ("alpha", ctypes.c_float), ("fbar", ctypes.c_float),
                ("unary", ctypes.c_void_p)]


class bp_sparse_potential(ctypes.Structure):
    """struct bp_sparse_potential (include/bp.h): host CSR arrays."""
    _fields_ = [("col_ptr", ctypes.POINTER(ctypes.c_int32)), ("row_idx", ctypes.POINTER(ctypes.c_int32)),
                ("val", ctypes.POINTER(ctypes.c_float)), ("fbar", ctypes.c_float)]


class bp_factor_type(ctypes.Structure):
    """struct bp_factor_type (include/bp.h): host tuple lists."""
    _fields_ = [("arity", ctypes.c_int32), ("n_tuples", ctypes.c_int32),
                ("tuples", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_float)),
                ("fbar", ctypes.c_float)]


class BPError(RuntimeError):
    def __init__(self, status, func, msg):
        super().__init__(f"{func} -> {status}: {msg}")
        self.status = status
        self.func = func


# name: (restype, argtypes)
_PROTOS = {
    "bp_init_grid": (_c_int, [ctypes.POINTER(_vp), _c_i32, _c_i32, _vp]),
    "bp_set_stream": (_c_int, [_vp, _vp]),
    "bp_set_potential": (_c_int, [_vp, _c_i32, _c_i32, _c_f, _c_f]),
    "bp_sparse_table_bytes": (_c_i64, [_vp, _c_i32, ctypes.POINTER(bp_sparse_potential)]),
    "bp_multiscale_workspace_bytes": (_c_i64, [_vp, _c_i32]),
    "bp_fg_init": (_c_int, [ctypes.POINTER(_vp), _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_i32),
                            ctypes.POINTER(_c_i32), _c_i32, ctypes.POINTER(bp_factor_type), _c_i32, _vp]),
    "bp_fg_set_stream": (_c_int, [_vp, _vp]),
    "bp_fg_workspace_bytes": (_c_i64, [_vp]),
    "bp_fg_attach_workspace": (_c_int, [_vp, _vp, _c_i64]),
    "bp_fg_set_unary": (_c_int, [_vp, _vp]),
    "bp_fg_reset_messages": (_c_int, [_vp]),
    "bp_fg_iterate": (_c_int, [_vp, _c_i32, _c_i32, _c_i32]),
    "bp_fg_beliefs": (_c_int, [_vp, _vp, _vp]),
    "bp_fg_get_messages": (_c_int, [_vp, _vp, _vp]),
    "bp_fg_destroy": (_c_int, [_vp]),
    "bp_iterate_multiscale": (_c_int, [_vp, _c_i32, _c_i32, ctypes.POINTER(_c_i32), _vp, _c_i64]),
    "bp_set_sparse_potentials": (_c_int, [_vp, _c_i32, ctypes.POINTER(bp_sparse_potential), _vp, _c_i64, _vp, _vp]),
    "bp_workspace_bytes": (_c_i64, [_vp]),
    "bp_attach_workspace": (_c_int, [_vp, _vp, _c_i64]),
    "bp_set_unary": (_c_int, [_vp, _vp]),
    "bp_reset_messages": (_c_int, [_vp]),
    "bp_set_sync_fusion": (_c_int, [_vp, _c_i32]),
    "bp_set_arithmetic": (_c_int, [_vp, _c_i32]),
    "bp_set_launch_tuning": (_c_int, [_vp, _c_i32, _c_i32]),
    "bp_message_stats": (_c_int, [_vp, _vp, _vp]),
    "bp_get_launch_tuning": (_c_int, [_vp, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "bp_autotune": (_c_int, [_vp, _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_f)]),
    "bp_iterate": (_c_int, [_vp, _c_i32, _c_i32, _c_i32]),
    "bp_solve_noalloc": (_c_int, [_vp, _c_i32, _c_i32, _c_i32, _c_i32, _c_f, _c_f, _c_i32, _c_i32, _c_i32, _vp, _vp,
                                  _vp]),
    "bp_iterate_dense": (_c_int, [_vp, _c_i32, _c_i32, _c_i32]),
    "bp_beliefs": (_c_int, [_vp, _vp]),
    "bp_map_labels": (_c_int, [_vp, _vp]),
    "bp_readout": (_c_int, [_vp, _vp, _vp]),
    "bp_get_messages": (_c_int, [_vp, _vp]),
    "bp_set_messages": (_c_int, [_vp, _vp]),
    "bp_grad_workspace_bytes": (_c_i64, [_vp, _c_i32, _c_i32]),
    "bp_forward_ckpt": (_c_int, [_vp, _c_i32, _c_i32, _vp, _c_i64]),
    "bp_backward": (_c_int, [_vp, _vp, _vp, _vp]),
    "bp_destroy": (_c_int, [_vp]),
    "bp_batch_init": (_c_int, [ctypes.POINTER(_vp), _c_i32, ctypes.POINTER(bp_grid_desc), _vp]),
    "bp_batch_set_stream": (_c_int, [_vp, _vp]),
    "bp_batch_workspace_bytes": (_c_i64, [_vp]),
    "bp_batch_attach_workspace": (_c_int, [_vp, _vp, _c_i64]),
    "bp_batch_reset_messages": (_c_int, [_vp]),
    "bp_batch_iterate": (_c_int, [_vp, _c_i32, _c_i32]),
    "bp_batch_set_graphs": (_c_int, [_vp, _c_i32]),
    "bp_batch_set_arithmetic": (_c_int, [_vp, _c_i32]),
    "bp_batch_set_plan": (_c_int, [_vp, ctypes.POINTER(_c_i32), _c_i32]),
    "bp_batch_get_plan": (_c_int, [_vp, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "bp_batch_set_streams": (_c_int, [_vp, _c_i32]),
    "bp_batch_get_streams": (_c_int, [_vp]),
    "bp_batch_autotune": (_c_int, [_vp, _c_i32, _c_i32, ctypes.POINTER(_c_f)]),
    "bp_batch_beliefs": (_c_int, [_vp, _vp]),
    "bp_batch_map_labels": (_c_int, [_vp, _vp]),
    "bp_batch_destroy": (_c_int, [_vp]),
    "bp_status_string": (ctypes.c_char_p, [_c_int]),
    "bp_last_error": (ctypes.c_char_p, []),
}

_lib = None


def header_symbols(path=HEADER):
    """Names of the functions include/bp.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bp_\w+)\s*\(", text)))


def lib():
    """Load libbp_hip.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    """Device address of a torch tensor (or an int address / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream, device=None):
    if stream is None:
        import torch
        return torch.cuda.current_stream(device).cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status, func):
    if status < 0:
        raise BPError(status, func, lib().bp_last_error().decode())
    return status


# ------------------------------------------------------------------ ABI ----

def bp_init_grid(H, W, stream=None):
    h = _vp()
    _check(lib().bp_init_grid(ctypes.byref(h), H, W, _stream(stream)), "bp_init_grid")
    return h.value


def bp_set_stream(handle, stream=None):
    _check(lib().bp_set_stream(handle, _stream(stream)), "bp_set_stream")


def bp_set_potential(handle, M, T, alpha, fbar):
    _check(lib().bp_set_potential(handle, M, T, alpha, fbar), "bp_set_potential")


def _sparse_types(types):
    """types: sequence of (col_ptr, row_idx, val, fbar) host arrays.  Returns the
    ctypes array and the contiguous numpy arrays it points into (keep alive)."""
    import numpy as np
    keep, arr = [], (bp_sparse_potential * len(types))()
    for k, (cp, ri, va, fb) in enumerate(types):
        cp = np.ascontiguousarray(cp, dtype=np.int32)
        ri = np.ascontiguousarray(ri, dtype=np.int32)
        va = np.ascontiguousarray(va, dtype=np.float32)
        keep += [cp, ri, va]
        arr[k].col_ptr = cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[k].row_idx = ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[k].val = va.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        arr[k].fbar = float(fb)
    return arr, keep


def bp_sparse_table_bytes(handle, types):
    arr, keep = _sparse_types(types)
    return _check(lib().bp_sparse_table_bytes(handle, len(types), arr), "bp_sparse_table_bytes")


def bp_set_sparse_potentials(handle, types, table, nbytes, type_h=None, type_v=None):
    arr, keep = _sparse_types(types)
    _check(lib().bp_set_sparse_potentials(handle, len(types), arr, _ptr(table), nbytes, _ptr(type_h), _ptr(type_v)),
           "bp_set_sparse_potentials")


def bp_multiscale_workspace_bytes(handle, levels):
    return _check(lib().bp_multiscale_workspace_bytes(handle, levels), "bp_multiscale_workspace_bytes")


def bp_iterate_multiscale(handle, mode, iters, ws, nbytes):
    arr = (_c_i32 * len(iters))(*iters)
    _check(lib().bp_iterate_multiscale(handle, mode, len(iters) - 1, arr, _ptr(ws), nbytes), "bp_iterate_multiscale")


def bp_fg_init(n_vars, M, factor_vars, factor_type, types, dense_tables=False, stream=None):
    """factor_vars: [n_factors, 3] int (third ignored for arity 2); types:
    sequence of (arity, tuples [C, arity], values [C], fbar)."""
    import numpy as np
    fv = np.ascontiguousarray(np.asarray(factor_vars, dtype=np.int32).reshape(-1, 3))
    ft = np.ascontiguousarray(np.asarray(factor_type, dtype=np.int32).reshape(-1))
    keep, arr = [fv, ft], (bp_factor_type * len(types))()
    for k, (arity, tuples, values, fbar) in enumerate(types):
        tu = np.ascontiguousarray(np.asarray(tuples, dtype=np.int32).reshape(-1, arity))
        va = np.ascontiguousarray(np.asarray(values, dtype=np.float32).reshape(-1))
        keep += [tu, va]
        arr[k].arity, arr[k].n_tuples, arr[k].fbar = arity, len(va), float(fbar)
        arr[k].tuples = tu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[k].val = va.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    h = _vp()
    _check(lib().bp_fg_init(ctypes.byref(h), n_vars, M, len(ft), fv.ctypes.data_as(ctypes.POINTER(_c_i32)),
                            ft.ctypes.data_as(ctypes.POINTER(_c_i32)), len(types), arr, int(bool(dense_tables)),
                            _stream(stream)), "bp_fg_init")
    return h.value


def bp_fg_set_stream(handle, stream=None):
    _check(lib().bp_fg_set_stream(handle, _stream(stream)), "bp_fg_set_stream")


def bp_fg_workspace_bytes(handle):
    return _check(lib().bp_fg_workspace_bytes(handle), "bp_fg_workspace_bytes")


def bp_fg_attach_workspace(handle, ws, nbytes):
    _check(lib().bp_fg_attach_workspace(handle, _ptr(ws), nbytes), "bp_fg_attach_workspace")


def bp_fg_set_unary(handle, g):
    _check(lib().bp_fg_set_unary(handle, _ptr(g)), "bp_fg_set_unary")


def bp_fg_reset_messages(handle):
    _check(lib().bp_fg_reset_messages(handle), "bp_fg_reset_messages")


def bp_fg_iterate(handle, mode, n_iters, dense=False):
    _check(lib().bp_fg_iterate(handle, mode, n_iters, int(bool(dense))), "bp_fg_iterate")


def bp_fg_beliefs(handle, beliefs=None, labels=None):
    _check(lib().bp_fg_beliefs(handle, _ptr(beliefs), _ptr(labels)), "bp_fg_beliefs")


def bp_fg_get_messages(handle, m=None, n=None):
    _check(lib().bp_fg_get_messages(handle, _ptr(m), _ptr(n)), "bp_fg_get_messages")


def bp_fg_destroy(handle):
    _check(lib().bp_fg_destroy(handle), "bp_fg_destroy")


def bp_workspace_bytes(handle):
    return _check(lib().bp_workspace_bytes(handle), "bp_workspace_bytes")


def bp_attach_workspace(handle, ws, nbytes=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    _check(lib().bp_attach_workspace(handle, _ptr(ws), nbytes), "bp_attach_workspace")


def bp_set_unary(handle, g):
    _check(lib().bp_set_unary(handle, _ptr(g)), "bp_set_unary")


def bp_reset_messages(handle):
    _check(lib().bp_reset_messages(handle), "bp_reset_messages")


def bp_set_sync_fusion(handle, enable):
    _check(lib().bp_set_sync_fusion(handle, 1 if enable else 0), "bp_set_sync_fusion")


def bp_set_arithmetic(handle, arith):
    _check(lib().bp_set_arithmetic(handle, arith), "bp_set_arithmetic")


def bp_message_stats(handle, max_change, non_finite):
    """max_change / non_finite: device pointers (or None)."""
    _check(lib().bp_message_stats(handle, _vp(max_change) if max_change else None,
                                  _vp(non_finite) if non_finite else None), "bp_message_stats")


def bp_set_launch_tuning(handle, layout, cap):
    _check(lib().bp_set_launch_tuning(handle, layout, cap), "bp_set_launch_tuning")


def bp_get_launch_tuning(handle):
    layout, cap = _c_i32(), _c_i32()
    _check(lib().bp_get_launch_tuning(handle, ctypes.byref(layout), ctypes.byref(cap)), "bp_get_launch_tuning")
    return layout.value, cap.value


def bp_autotune(handle, mode, schedule, trial_iters):
    best = _c_f()
    _check(lib().bp_autotune(handle, mode, schedule, trial_iters, ctypes.byref(best)), "bp_autotune")
    return best.value


def bp_iterate(handle, mode, n_iters, schedule):
    _check(lib().bp_iterate(handle, mode, n_iters, schedule), "bp_iterate")


def bp_solve_noalloc(g, H, W, M, T, alpha, fbar, mode, n_iters, schedule, beliefs, labels, stream=None):
    """stream: a torch stream, a raw hipStream_t address (int) or None for
    torch's current stream on g's device."""
    dev = g.device if hasattr(g, "device") else None
    _check(lib().bp_solve_noalloc(_ptr(g), H, W, M, T, alpha, BP_FBAR_TIED if fbar is None else fbar, mode,
                                  n_iters, schedule, _ptr(beliefs), _ptr(labels), _stream(stream, dev)),
           "bp_solve_noalloc")


def bp_iterate_dense(handle, mode, n_iters, schedule):
    _check(lib().bp_iterate_dense(handle, mode, n_iters, schedule), "bp_iterate_dense")


def bp_beliefs(handle, out):
    _check(lib().bp_beliefs(handle, _ptr(out)), "bp_beliefs")


def bp_map_labels(handle, out):
    _check(lib().bp_map_labels(handle, _ptr(out)), "bp_map_labels")


def bp_readout(handle, beliefs, labels):
    _check(lib().bp_readout(handle, _ptr(beliefs), _ptr(labels)), "bp_readout")


def bp_get_messages(handle, dst):
    _check(lib().bp_get_messages(handle, _ptr(dst)), "bp_get_messages")


def bp_set_messages(handle, src):
    _check(lib().bp_set_messages(handle, _ptr(src)), "bp_set_messages")


def bp_grad_workspace_bytes(handle, n_iters, ckpt_every):
    return _check(lib().bp_grad_workspace_bytes(handle, n_iters, ckpt_every), "bp_grad_workspace_bytes")


def bp_forward_ckpt(handle, n_iters, ckpt_every, gws, nbytes=None):
    if nbytes is None:
        nbytes = gws.numel() * gws.element_size()
    _check(lib().bp_forward_ckpt(handle, n_iters, ckpt_every, _ptr(gws), nbytes), "bp_forward_ckpt")


def bp_backward(handle, dL_db, dtheta, dalpha):
    _check(lib().bp_backward(handle, _ptr(dL_db), _ptr(dtheta), _ptr(dalpha)), "bp_backward")


def bp_destroy(handle):
    _check(lib().bp_destroy(handle), "bp_destroy")


def bp_status_string(status):
    return lib().bp_status_string(status).decode()


def bp_last_error():
    return lib().bp_last_error().decode()


# ---------------------------------------------------------------- batch ----

def bp_batch_init(descs, stream=None):
    """descs: sequence of bp_grid_desc (unary = device address)."""
    arr = (bp_grid_desc * len(descs))(*descs)
    h = _vp()
    _check(lib().bp_batch_init(ctypes.byref(h), len(descs), arr, _stream(stream)), "bp_batch_init")
    return h.value


def bp_batch_set_stream(handle, stream=None):
    _check(lib().bp_batch_set_stream(handle, _stream(stream)), "bp_batch_set_stream")


def bp_batch_workspace_bytes(handle):
    return _check(lib().bp_batch_workspace_bytes(handle), "bp_batch_workspace_bytes")


def bp_batch_attach_workspace(handle, ws, nbytes=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    _check(lib().bp_batch_attach_workspace(handle, _ptr(ws), nbytes), "bp_batch_attach_workspace")


def bp_batch_reset_messages(handle):
    _check(lib().bp_batch_reset_messages(handle), "bp_batch_reset_messages")


def bp_batch_iterate(handle, mode, n_iters):
    _check(lib().bp_batch_iterate(handle, mode, n_iters), "bp_batch_iterate")


def bp_batch_set_graphs(handle, enable):
    _check(lib().bp_batch_set_graphs(handle, int(bool(enable))), "bp_batch_set_graphs")


def bp_batch_set_arithmetic(handle, arith):
    _check(lib().bp_batch_set_arithmetic(handle, arith), "bp_batch_set_arithmetic")


BP_BATCH_CLASSES = 5


def bp_batch_set_plan(handle, passes, grid_blocks):
    arr = (_c_i32 * BP_BATCH_CLASSES)(*passes)
    _check(lib().bp_batch_set_plan(handle, arr, grid_blocks), "bp_batch_set_plan")


def bp_batch_get_plan(handle):
    arr = (_c_i32 * BP_BATCH_CLASSES)()
    g = _c_i32()
    _check(lib().bp_batch_get_plan(handle, arr, ctypes.byref(g)), "bp_batch_get_plan")
    return list(arr), g.value


def bp_batch_set_streams(handle, n_streams):
    _check(lib().bp_batch_set_streams(handle, n_streams), "bp_batch_set_streams")


def bp_batch_get_streams(handle):
    r = lib().bp_batch_get_streams(handle)
    _check(min(r, 0), "bp_batch_get_streams")
    return r


def bp_batch_autotune(handle, mode, trial_iters):
    best = _c_f()
    _check(lib().bp_batch_autotune(handle, mode, trial_iters, ctypes.byref(best)), "bp_batch_autotune")
    return best.value


def bp_batch_beliefs(handle, out):
    _check(lib().bp_batch_beliefs(handle, _ptr(out)), "bp_batch_beliefs")


def bp_batch_map_labels(handle, out):
    _check(lib().bp_batch_map_labels(handle, _ptr(out)), "bp_batch_map_labels")


def bp_batch_destroy(handle):
    _check(lib().bp_batch_destroy(handle), "bp_batch_destroy")
