"""ctypes declarations of libgs.so (the C ABI in include/gs.h).

Only argument marshalling lives here.  The library is loaded from the
package directory; if it is missing, every entry point raises -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK = 0
GS_ERR_INVALID_ARG = 1
GS_ERR_UNSUPPORTED = 2
GS_ERR_HIP = 3

GS_MAX_VIEWS = 64
GS_CAMERA_FLOATS = 20

GS_CUTOFF_3SIGMA = 1 << 0
GS_FUSED_L1 = 1 << 1
GS_ACCUMULATE_GRADS = 1 << 2
GS_PERSISTENT = 1 << 3
GS_SPLAT_BWD = 1 << 4
GS_RADIX_BIN = 1 << 5

GS_WS_RECORDS = 0
GS_WS_RECTS = 1
GS_WS_TILES_TOUCHED = 2
GS_WS_PAIR_OFFSETS = 3
GS_WS_SORTED_KEYS = 4
GS_WS_SORTED_VALS = 5
GS_WS_SORTED_RECS = 6
GS_WS_RANGES = 7

F_OVERFLOW, F_NONFINITE, F_PAIRS, F_VISIBLE = 0, 1, 2, 3
F_PAIRS_WANTED = 6

vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
f32 = ctypes.c_float
f64 = ctypes.c_double
u32 = ctypes.c_uint32
sz = ctypes.c_size_t


class GsGaussians(ctypes.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logits", vp),
                ("sh", vp), ("n", i64), ("sh_degree", i32)]


class GsGaussianGrads(ctypes.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logits", vp),
                ("sh", vp)]


class GsRasterCfg(ctypes.Structure):
    _fields_ = [("tile_w", i32), ("tile_h", i32), ("chunk", i32), ("lds_batch", i32),
                ("flags", u32), ("lambda_depth", f32)]


class GsPlan(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_uint64 * 640)]


class GsParamGroup(ctypes.Structure):
    _fields_ = [("p", vp), ("g", vp), ("m", vp), ("v", vp), ("n", i64), ("lr", f32),
                ("opacity_reg", i32)]


class GsViewGather(ctypes.Structure):
    _fields_ = [("pool_cams", vp), ("pool_rgb", vp), ("pool_depth", vp), ("sel", vp),
                ("n_pool", i32)]


class GsIteration(ctypes.Structure):
    _fields_ = [("plan", ctypes.POINTER(GsPlan)), ("ws", vp), ("gaussians", GsGaussians),
                ("cams_dev", vp), ("color", vp), ("depth", vp), ("T_final", vp), ("last", vp),
                ("target_rgb", vp), ("target_depth", vp), ("loss_per_view", vp),
                ("dL_dcolor", vp), ("dL_ddepth", vp), ("grads", GsGaussianGrads),
                ("dL_dpose", vp), ("adam_groups", ctypes.POINTER(GsParamGroup)),
                ("n_adam_groups", i32), ("step_dev", vp), ("beta1", f64), ("beta2", f64),
                ("eps", f64), ("lambda_o", f64), ("reg_count", i64), ("lambda_ssim", f64),
                ("loss_grad_color", vp), ("loss_grad_depth", vp),
                ("gather", ctypes.POINTER(GsViewGather))]


class GsScheduler(ctypes.Structure):
    _fields_ = [("r", ctypes.POINTER(i32)), ("l", ctypes.POINTER(ctypes.c_double)),
                ("capacity", i32), ("count", i32), ("r0", i32), ("d", i32),
                ("refills", i64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "gs_plan_init": (i32, [ctypes.POINTER(GsPlan), i64, i32, i32, ctypes.POINTER(i32),
                           ctypes.POINTER(GsRasterCfg), i64]),
    "gs_workspace_size": (sz, [ctypes.POINTER(GsPlan)]),
    "gs_plan_total_pixels": (i64, [ctypes.POINTER(GsPlan)]),
    "gs_plan_pixel_offset": (i64, [ctypes.POINTER(GsPlan), i32]),
    "gs_plan_total_tiles": (i64, [ctypes.POINTER(GsPlan)]),
    "gs_plan_ws_offset": (i64, [ctypes.POINTER(GsPlan), i32]),
    "gs_flags_ptr": (vp, [ctypes.POINTER(GsPlan), vp]),
    "gs_preprocess": (i32, [ctypes.POINTER(GsPlan), ctypes.POINTER(GsGaussians), vp, vp, vp]),
    "gs_bin_sort": (i32, [ctypes.POINTER(GsPlan), vp, vp]),
    "gs_render_fwd": (i32, [ctypes.POINTER(GsPlan), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "gs_render_bwd": (i32, [ctypes.POINTER(GsPlan), ctypes.POINTER(GsGaussians), vp, vp, vp, vp,
                            vp, vp, vp, vp, vp, vp, ctypes.POINTER(GsGaussianGrads), vp, vp]),
    "gs_render_loss": (i32, [ctypes.POINTER(GsPlan), vp, vp, vp, vp, vp, f64, vp, vp, vp, vp]),
    "gs_render_bwd_raster": (i32, [ctypes.POINTER(GsPlan), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   vp, vp]),
    "gs_project_bwd": (i32, [ctypes.POINTER(GsPlan), ctypes.POINTER(GsGaussians), vp, vp,
                             ctypes.POINTER(GsGaussianGrads), vp, vp]),
    "gs_adam_step": (i32, [ctypes.POINTER(GsParamGroup), i32, i32, f64, f64, f64, f64, i64, vp,
                           vp]),
    "gs_pose_retract": (i32, [vp, vp, vp, i32, vp]),
    "gs_pose_tangent_vjp": (i32, [vp, vp, vp, i32, vp]),
    "gs_grad_stats": (i32, [ctypes.POINTER(GsPlan), vp, vp, vp, vp]),
    "gs_densify_tmp_bytes": (sz, [i64]),
    "gs_densify_prune": (i32, [ctypes.POINTER(GsGaussians), ctypes.POINTER(GsGaussianGrads),
                               ctypes.POINTER(GsGaussianGrads), vp, vp, vp, f32, f32, f32, f32,
                               ctypes.POINTER(GsGaussianGrads), ctypes.POINTER(GsGaussianGrads),
                               ctypes.POINTER(GsGaussianGrads), i64, vp, vp, vp]),
    "gs_sort_tmp_bytes": (sz, [i64]),
    "gs_sort_pairs": (i32, [vp, vp, i64, i32, vp, vp]),
    "gs_sort_pairs_noalloc": (i32, [vp, vp, i64, i32, vp]),
    "gs_spatial_order_tmp_bytes": (sz, [i64]),
    "gs_spatial_order": (i32, [vp, i64, vp, vp, vp]),
    "gs_permute_gaussians": (i32, [ctypes.POINTER(GsGaussians), vp,
                                   ctypes.POINTER(GsGaussianGrads), vp]),
    "gs_gather_views": (i32, [ctypes.POINTER(GsPlan), ctypes.POINTER(GsViewGather), vp, vp, vp,
                              vp]),
    "gs_iteration_enqueue": (i32, [ctypes.POINTER(GsIteration), vp]),
    "gs_graph_create": (i32, [ctypes.POINTER(GsIteration), vp, ctypes.POINTER(vp)]),
    "gs_graph_launch": (i32, [vp, vp]),
    "gs_graph_destroy": (i32, [vp]),
    "gs_graph_time": (i32, [vp, vp, i32, i32, ctypes.POINTER(f32)]),
    "gs_iteration_time_marks": (i32, [ctypes.POINTER(GsIteration), vp, i32, i32,
                                      ctypes.POINTER(f32)]),
    "gs_sched_init": (i32, [ctypes.POINTER(GsScheduler), ctypes.POINTER(i32),
                            ctypes.POINTER(ctypes.c_double), i32, i32, i32]),
    "gs_sched_add_keyframe": (i32, [ctypes.POINTER(GsScheduler), ctypes.POINTER(i32)]),
    "gs_sched_select": (i32, [ctypes.POINTER(GsScheduler), i32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "gs_sched_report": (i32, [ctypes.POINTER(GsScheduler), i32, ctypes.c_double]),
    "gs_sched_last_error": (ctypes.c_char_p, []),
    "gs_status_string": (ctypes.c_char_p, [i32]),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_version": (i32, []),
}

_lib = None


class GsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load libgs.so; raise loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != GS_OK:
        L = lib()
        raise GsError(status, f"{L.gs_status_string(status).decode()}: {L.gs_last_error().decode()}")
