"""RaDe-GS rasterizer (arXiv 2406.01467) for AMD Instinct MI355X.

The rasterizer projects 3D Gaussians to splats, bins and depth-sorts them per
screen tile and alpha-blends colour, the paper's planar per-splat depth and
its normal into colour / depth (expected and median) / normal / alpha maps,
forward and backward.  The compute path is the HIP library librade.so
(include/rade.h); this package binds it for PyTorch tensors.
"""
from ._lib import Settings, RadeError, SPLAT_DTYPE  # noqa: F401

__all__ = ["Settings", "RadeError", "SPLAT_DTYPE", "Rasterizer", "render"]


def __getattr__(name):
    if name in ("Rasterizer", "render", "Maps", "ForwardState"):
        from . import raster as _r
        return getattr(_r, name)
    raise AttributeError(name)
