"""The C ABI without a GPU: the library loads, exports every function
include/bp.h declares, and rejects bad arguments before touching a device."""
import ctypes

import pytest

from paper_1010_0012_amd import _lib as L


def test_exports_every_declared_symbol():
    names = L.header_symbols()
    assert "bp_iterate" in names and "bp_set_potential" in names
    lib = L.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L._PROTOS) >= set(names), set(names) - set(L._PROTOS)


def test_status_strings():
    for code in (L.BP_OK, L.BP_EINVAL, L.BP_ESTATE, L.BP_ENOMEM, L.BP_EHIP, L.BP_EUNSUPPORTED):
        assert L.bp_status_string(code).startswith("BP_")
    assert L.bp_status_string(-99) == "unknown status"


def test_host_side_argument_checks():
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.bp_init_grid(None, 4, 4, None) == L.BP_EINVAL
    assert lib.bp_init_grid(ctypes.byref(h), 0, 4, None) == L.BP_EINVAL
    assert "both sides" in L.bp_last_error()
    assert lib.bp_init_grid(ctypes.byref(h), 4, -1, None) == L.BP_EINVAL
    assert lib.bp_init_grid(ctypes.byref(h), 1 << 15, 1 << 15, None) == L.BP_EINVAL
    assert lib.bp_set_potential(None, 8, 2, 1.0, 0.1) == L.BP_EINVAL
    assert lib.bp_iterate(None, 0, 1, 0) == L.BP_EINVAL
    assert lib.bp_workspace_bytes(None) == L.BP_EINVAL
    assert lib.bp_beliefs(None, None) == L.BP_EINVAL
    assert lib.bp_readout(None, None, None) == L.BP_EINVAL
    assert lib.bp_readout(None, ctypes.c_void_p(16), None) == L.BP_EINVAL
    assert lib.bp_set_launch_tuning(None, 0, -1) == L.BP_EINVAL
    lay, cap = ctypes.c_int32(), ctypes.c_int32()
    assert lib.bp_get_launch_tuning(None, ctypes.byref(lay), ctypes.byref(cap)) == L.BP_EINVAL
    assert lib.bp_autotune(None, 0, 0, 2, None) == L.BP_EINVAL
    assert lib.bp_batch_set_arithmetic(None, 1) == L.BP_EINVAL
    assert lib.bp_destroy(None) == L.BP_OK


def test_no_device_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.lib().bp_init_grid(ctypes.byref(h), 4, 4, None) == L.BP_EHIP
    assert h.value is None
