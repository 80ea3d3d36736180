"""MI355X-native (gfx950) differentiable 3D Gaussian-splatting rasterizer:
the per-iteration hot path of the CaRtGS mapping back-end (preprocess, tile
binning into per-tile depth-sorted lists, LDS-staged compositing,
back-to-front backward with camera-tangent gradients, Adam), behind the C
ABI of include/gs.h.  This package only marshals arguments to libgs.so."""
from . import _lib
from .sched import KeyframeScheduler
from .raster import (Frame, Gaussians, Iteration, KeyframePool, Mapper, Plan, Rasterizer,
                     adam_groups, adam_step, bin_sort, cameras_tensor, densify_prune, grad_stats,
                     permute, pose_retract, pose_tangent_vjp, preprocess, project_bwd, rasterize,
                     render_bwd, render_bwd_raster, render_fwd, render_loss, required_pairs,
                     sort_pairs, sort_pairs_noalloc, spatial_order)

__all__ = ["KeyframeScheduler", "Frame", "Gaussians", "Iteration", "KeyframePool", "Mapper",
           "Plan", "Rasterizer", "adam_groups", "adam_step", "bin_sort", "cameras_tensor",
           "densify_prune", "grad_stats", "permute", "pose_retract", "pose_tangent_vjp",
           "preprocess", "project_bwd", "rasterize", "render_bwd", "render_bwd_raster",
           "render_fwd", "render_loss", "required_pairs", "sort_pairs", "sort_pairs_noalloc",
           "spatial_order"]
