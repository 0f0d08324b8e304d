"""Exact O(mM) belief propagation for truncated-potential grid MRFs on MI355X.

The compute lives in libbp_hip.so (hand-written HIP for gfx950, C ABI in
include/bp.h); this package is its Python binding.  Importing the package
does not load the library; the first call does, and fails loudly if it has
not been built.
"""
__all__ = ["Grid", "lib"]


def __getattr__(name):
    if name == "Grid":
        from .grid import Grid
        return Grid
    if name == "lib":
        from . import _lib
        return _lib
    raise AttributeError(name)
