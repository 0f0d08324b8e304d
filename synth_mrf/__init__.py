"""Seeded synthetic stereo-like grid MRF inputs.

This module only draws inputs (images, disparity maps, unary tables and the
per-workload parameter sets).  It holds none of the belief-propagation
arithmetic, so both the FP64 oracle and the GPU path may import it.

The paper's experiment (Sec. 6) runs on the Tsukuba stereo pair, which is not
available here; the generators below stand in for it with the same structure:
a textured left image, a piecewise-constant or piecewise-planar disparity map,
a right image made by shifting the left one by that disparity plus Gaussian
noise, and the absolute-intensity-difference unary potential of Sec. 6.
"""
from .stereo import (  # noqa: F401
    GridConfig,
    CONFIGS,
    BatchInstance,
    make_stereo,
    make_config,
    make_batch_configs,
    make_batch_instance,
    random_unary,
    sha256_of,
)
from .factor import FactorGridSpec, make_factor_grid, smoothness_triples  # noqa: F401,E402
