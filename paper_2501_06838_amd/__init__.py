"""MI355X (gfx950) scale-aware differentiable 2D Gaussian rasterizer of GSASR
(arXiv 2501.06838, Sec. 3.1, Eq. 1-4, Algorithm 1).

The compute path is the HIP library ``libgsraster.so`` (C ABI in
include/gs_raster.h); this package only marshals arguments to it.
"""
from ._native import (GS_FLAG_ATOMIC_GRADS, GS_FLAG_ELLIPSE, GS_FLAG_PERSISTENT,  # noqa: F401
                      GS_FLAG_PIXEL_CENTER, GS_FLAG_RADIX_SORT)
from .raster import GSRasterize, RasterPlan, StepGraph, l1_loss_grad, rasterize  # noqa: F401

__all__ = ["GSRasterize", "RasterPlan", "StepGraph", "rasterize", "l1_loss_grad",
           "GS_FLAG_PERSISTENT", "GS_FLAG_ATOMIC_GRADS", "GS_FLAG_RADIX_SORT",
           "GS_FLAG_PIXEL_CENTER", "GS_FLAG_ELLIPSE"]
