"""MI355X-native (gfx950) differentiable 3D Gaussian-splatting rasterizer:
the per-iteration hot path of the CaRtGS mapping back-end (preprocess, tile
binning with a device radix sort, LDS-staged compositing, back-to-front
backward with camera-tangent gradients, Adam), behind the C ABI of
include/gs.h.  This package only marshals arguments to libgs.so."""
from . import _lib
from .sched import KeyframeScheduler
from .raster import (Frame, Gaussians, densify_prune, grad_stats, Iteration, Plan, adam_groups, adam_step, bin_sort,
                     cameras_tensor, preprocess, project_bwd, rasterize, render_bwd,
                     render_bwd_raster, render_fwd, render_loss, required_pairs,
                     sort_pairs)

__all__ = ["KeyframeScheduler", "densify_prune", "grad_stats", "Frame", "Gaussians", "Iteration", "Plan", "adam_groups", "adam_step", "bin_sort",
           "cameras_tensor", "preprocess", "project_bwd", "rasterize", "render_bwd",
           "render_bwd_raster", "render_fwd", "render_loss", "required_pairs", "sort_pairs"]
