"""MI355X (gfx950) ADER-WENO zone update for the 2D/3D compressible Euler equations.

The product is the C ABI in ``include/hog.h`` implemented by ``libhog.so``
(hand-written HIP kernels); :mod:`paper_2211_13295_amd.hog` is a thin ctypes
binding that uses PyTorch only for device memory and streams.
"""
from .hog import Grid, HogError, load, make_config, workspace_size  # noqa: F401

__all__ = ["Grid", "HogError", "load", "make_config", "workspace_size"]
