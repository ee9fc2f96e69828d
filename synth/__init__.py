"""Seeded synthetic interferometer datasets for the stacking tests and benchmark.

This package is shared by the FP64 CPU oracle tests and the GPU path.  It only
models the *sky and the instrument* (antenna layout, earth-rotation uvw, a
spectral-line source, noise, flags and weights); it holds none of the stacking
method's arithmetic (no phase re-centring, no rest-frame rebinning, no
gridding).  Random numbers are drawn here and handed to both sides as inputs.
"""
from .configs import CONFIGS, config, grid_for
from .generate import Target, batch_stack_sizes, make_target, make_targets, make_grid, radec_of_offset
from .pool import make_pool, pool_targets

__all__ = ["CONFIGS", "config", "grid_for", "Target", "batch_stack_sizes", "make_target", "make_targets",
           "make_grid", "radec_of_offset", "make_pool", "pool_targets"]
