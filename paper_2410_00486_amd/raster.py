"""Python binding of the gfx950 rasterizer: plans, workspaces, the five
entry points of a mapping iteration, HIP graphs, and a torch.autograd
Function with the camera-tangent gradient.

PyTorch provides device memory and the current stream; every step of the
path runs in libgs.so.  Nothing here computes pixels or gradients.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

_DEFAULT_TILE = (16, 16)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype=torch.float32):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


class Plan:
    """Host-side execution plan (sizes, tile grid, workspace layout)."""

    def __init__(self, n: int, sh_degree: int, view_wh: Sequence[Tuple[int, int]],
                 tile=_DEFAULT_TILE, lds_batch: int = 256, chunk: int = 2, flags: int = 0,
                 lambda_depth: float = 0.1, pair_capacity: int = 1 << 20):
        self.n, self.sh_degree = int(n), int(sh_degree)
        self.view_wh = [(int(w), int(h)) for (w, h) in view_wh]
        self.tile = (int(tile[0]), int(tile[1]))
        self.lds_batch, self.chunk, self.flags = int(lds_batch), int(chunk), int(flags)
        self.lambda_depth = float(lambda_depth)
        self.pair_capacity = int(pair_capacity)
        self.c = L.GsPlan()
        self.cfg = L.GsRasterCfg(self.tile[0], self.tile[1], self.chunk, self.lds_batch,
                                 self.flags, self.lambda_depth)
        wh = (ctypes.c_int32 * (2 * len(self.view_wh)))(*[v for p in self.view_wh for v in p])
        L.check(L.lib().gs_plan_init(ctypes.byref(self.c), self.n, self.sh_degree,
                                     len(self.view_wh), wh, ctypes.byref(self.cfg),
                                     self.pair_capacity))
        self.ws_bytes = int(L.lib().gs_workspace_size(ctypes.byref(self.c)))
        self.total_pixels = int(L.lib().gs_plan_total_pixels(ctypes.byref(self.c)))
        self.total_tiles = int(L.lib().gs_plan_total_tiles(ctypes.byref(self.c)))
        self.pixel_offsets = [int(L.lib().gs_plan_pixel_offset(ctypes.byref(self.c), v))
                              for v in range(len(self.view_wh))]

    @property
    def n_views(self):
        return len(self.view_wh)

    def replace(self, **kw) -> "Plan":
        args = dict(n=self.n, sh_degree=self.sh_degree, view_wh=self.view_wh, tile=self.tile,
                    lds_batch=self.lds_batch, chunk=self.chunk, flags=self.flags,
                    lambda_depth=self.lambda_depth, pair_capacity=self.pair_capacity)
        args.update(kw)
        return Plan(**args)

    def ws_offset(self, region: int) -> int:
        return int(L.lib().gs_plan_ws_offset(ctypes.byref(self.c), region))

    def new_workspace(self, device="cuda") -> torch.Tensor:
        # zero-filled: a whole iteration relies on the per-tile counters being
        # zero before its first projection (later binnings leave them so)
        ws = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        if ws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        return ws

    def flags_of(self, ws: torch.Tensor) -> np.ndarray:
        """Device flags (synchronises the current stream)."""
        ptr = L.lib().gs_flags_ptr(ctypes.byref(self.c), _ptr(ws))
        off = ptr - ws.data_ptr()
        return ws[off:off + 64].view(torch.int32).cpu().numpy()

    def region(self, ws: torch.Tensor, region: int, dtype, count: int) -> torch.Tensor:
        off = self.ws_offset(region)
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return ws[off:off + nbytes].view(dtype)

    def split_views(self, img: torch.Tensor, channels: int = 1) -> List[torch.Tensor]:
        out = []
        for (w, h), off in zip(self.view_wh, self.pixel_offsets):
            out.append(img[channels * off:channels * (off + w * h)].view(channels, h, w)
                       if channels > 1 else img[off:off + w * h].view(h, w))
        return out


class Gaussians:
    """Device parameters (contiguous float32 CUDA tensors)."""

    FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree):
        self.means = _need(means, "means")
        self.log_scales = _need(log_scales, "log_scales")
        self.quats = _need(quats, "quats")
        self.opacity_logits = _need(opacity_logits, "opacity_logits")
        self.sh = _need(sh, "sh")
        self.sh_degree = int(sh_degree)
        n = self.means.shape[0]
        k = (self.sh_degree + 1) ** 2
        if (self.means.shape != (n, 3) or self.log_scales.shape != (n, 3)
                or self.quats.shape != (n, 4) or self.opacity_logits.numel() != n
                or self.sh.numel() != n * k * 3):
            raise ValueError("parameter shapes must be [n,3], [n,3], [n,4], [n], [n,(deg+1)^2,3]")

    @property
    def n(self):
        return int(self.means.shape[0])

    def c(self) -> L.GsGaussians:
        return L.GsGaussians(self.means.data_ptr(), self.log_scales.data_ptr(),
                             self.quats.data_ptr(), self.opacity_logits.data_ptr(),
                             self.sh.data_ptr(), self.n, self.sh_degree)

    def tensors(self):
        return [getattr(self, f) for f in self.FIELDS]

    @staticmethod
    def from_scene(scene, device="cuda") -> "Gaussians":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats),
                         t(scene.opacity_logits),
                         t(scene.sh.reshape(scene.n, (scene.sh_degree + 1) ** 2, 3)),
                         scene.sh_degree)

    def zeros_like(self) -> "Gaussians":
        return Gaussians(*[torch.zeros_like(x) for x in self.tensors()], self.sh_degree)

    def grads_c(self) -> L.GsGaussianGrads:
        return L.GsGaussianGrads(*[x.data_ptr() for x in self.tensors()])


def cameras_tensor(cams, device="cuda") -> torch.Tensor:
    """[V, 20] float32 device camera records from objects with as_array()."""
    arr = np.stack([np.asarray(c.as_array() if hasattr(c, "as_array") else c, np.float32)
                    for c in cams])
    if arr.shape[1] != L.GS_CAMERA_FLOATS:
        raise ValueError("camera records must have 20 floats")
    return torch.from_numpy(arr).to(device).contiguous()


class Frame:
    """Forward outputs of one iteration, concatenated over views."""

    def __init__(self, plan: Plan, device="cuda"):
        P = plan.total_pixels
        self.color = torch.empty(3 * P, dtype=torch.float32, device=device)
        self.depth = torch.empty(P, dtype=torch.float32, device=device)
        self.T_final = torch.empty(P, dtype=torch.float32, device=device)
        self.last = torch.empty(P, dtype=torch.int32, device=device)
        self.loss = torch.zeros(plan.n_views, dtype=torch.float32, device=device)


# ---------------------------------------------------------------- entry points

def _check_cams(plan: Plan, cams: torch.Tensor):
    _need(cams, "cams")
    if cams.numel() != plan.n_views * L.GS_CAMERA_FLOATS:
        raise ValueError(f"cams must hold {plan.n_views} x {L.GS_CAMERA_FLOATS} floats")


def _check_ws(plan: Plan, ws: torch.Tensor):
    if not (ws.is_cuda and ws.numel() >= plan.ws_bytes):
        raise ValueError("workspace too small for the plan")


def preprocess(plan: Plan, ws: torch.Tensor, g: Gaussians, cams: torch.Tensor, stream=None):
    _check_cams(plan, cams)
    _check_ws(plan, ws)
    if g.n != plan.n or g.sh_degree != plan.sh_degree:
        raise ValueError("Gaussians do not match the plan")
    gc = g.c()
    L.check(L.lib().gs_preprocess(ctypes.byref(plan.c), ctypes.byref(gc), _ptr(cams), _ptr(ws),
                                  _stream(stream)))


def bin_sort(plan: Plan, ws: torch.Tensor, stream=None):
    _check_ws(plan, ws)
    L.check(L.lib().gs_bin_sort(ctypes.byref(plan.c), _ptr(ws), _stream(stream)))


def _check_img(t, n, name):
    if t is not None and (not t.is_cuda or t.numel() != n or not t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA tensor of {n} elements")


def render_fwd(plan: Plan, ws: torch.Tensor, cams: torch.Tensor, out: Frame,
               target_rgb=None, target_depth=None, stream=None):
    _check_cams(plan, cams)
    _check_ws(plan, ws)
    P = plan.total_pixels
    for t, n, name in ((out.color, 3 * P, "color"), (out.depth, P, "depth"),
                       (out.T_final, P, "T_final"), (out.last, P, "last"),
                       (target_rgb, 3 * P, "target_rgb"), (target_depth, P, "target_depth")):
        _check_img(t, n, name)
    L.check(L.lib().gs_render_fwd(
        ctypes.byref(plan.c), _ptr(ws), _ptr(cams), _ptr(out.color), _ptr(out.depth),
        _ptr(out.T_final), _ptr(out.last), _ptr(target_rgb), _ptr(target_depth),
        _ptr(out.loss) if target_rgb is not None else None, _stream(stream)))


def render_bwd(plan: Plan, ws: torch.Tensor, g: Gaussians, cams: torch.Tensor, fr: Frame,
               grads: Gaussians, dL_dcolor=None, dL_ddepth=None, target_rgb=None,
               target_depth=None, dL_dpose=None, stream=None):
    _check_cams(plan, cams)
    _check_ws(plan, ws)
    P = plan.total_pixels
    for t, n, name in ((dL_dcolor, 3 * P, "dL_dcolor"), (dL_ddepth, P, "dL_ddepth"),
                       (target_rgb, 3 * P, "target_rgb"), (target_depth, P, "target_depth")):
        _check_img(t, n, name)
    if dL_dpose is not None and dL_dpose.numel() != 6 * plan.n_views:
        raise ValueError("dL_dpose must hold n_views x 6 floats")
    for a, b in zip(g.tensors(), grads.tensors()):
        if a.shape != b.shape:
            raise ValueError("gradient buffers must match the parameter shapes")
    gc = g.c()
    out = grads.grads_c()
    L.check(L.lib().gs_render_bwd(
        ctypes.byref(plan.c), ctypes.byref(gc), _ptr(cams), _ptr(ws), _ptr(fr.color),
        _ptr(fr.depth), _ptr(fr.T_final), _ptr(fr.last), _ptr(dL_dcolor), _ptr(dL_ddepth),
        _ptr(target_rgb), _ptr(target_depth), ctypes.byref(out), _ptr(dL_dpose),
        _stream(stream)))


def render_loss(plan: Plan, ws: torch.Tensor, fr: Frame, target_rgb, target_depth=None,
                lambda_ssim: float = 0.2, dL_dcolor=None, dL_ddepth=None, stream=None):
    """Eq. (9) loss per view (into fr.loss) and its image gradients."""
    _check_ws(plan, ws)
    P = plan.total_pixels
    if dL_dcolor is None:
        dL_dcolor = torch.empty(3 * P, dtype=torch.float32, device=ws.device)
    if dL_ddepth is None:
        dL_ddepth = torch.empty(P, dtype=torch.float32, device=ws.device)
    for t, n, name in ((target_rgb, 3 * P, "target_rgb"), (target_depth, P, "target_depth"),
                       (dL_dcolor, 3 * P, "dL_dcolor"), (dL_ddepth, P, "dL_ddepth")):
        _check_img(t, n, name)
    L.check(L.lib().gs_render_loss(ctypes.byref(plan.c), _ptr(ws), _ptr(fr.color), _ptr(fr.depth),
                                   _ptr(target_rgb), _ptr(target_depth), float(lambda_ssim),
                                   _ptr(dL_dcolor), _ptr(dL_ddepth), _ptr(fr.loss),
                                   _stream(stream)))
    return dL_dcolor, dL_ddepth


def render_bwd_raster(plan: Plan, ws: torch.Tensor, cams: torch.Tensor, fr: Frame,
                      dL_dcolor=None, dL_ddepth=None, target_rgb=None, target_depth=None,
                      stream=None):
    """Stage a5 only: per-pair partial gradients into the workspace."""
    _check_cams(plan, cams)
    _check_ws(plan, ws)
    L.check(L.lib().gs_render_bwd_raster(
        ctypes.byref(plan.c), _ptr(ws), _ptr(cams), _ptr(fr.color), _ptr(fr.depth),
        _ptr(fr.T_final), _ptr(fr.last), _ptr(dL_dcolor), _ptr(dL_ddepth), _ptr(target_rgb),
        _ptr(target_depth), _stream(stream)))


def project_bwd(plan: Plan, ws: torch.Tensor, g: Gaussians, cams: torch.Tensor,
                grads: Gaussians, dL_dpose=None, stream=None):
    """Stage a6 only: per-Gaussian reduction and chain rule."""
    _check_cams(plan, cams)
    _check_ws(plan, ws)
    gc = g.c()
    out = grads.grads_c()
    L.check(L.lib().gs_project_bwd(ctypes.byref(plan.c), ctypes.byref(gc), _ptr(cams), _ptr(ws),
                                   ctypes.byref(out), _ptr(dL_dpose), _stream(stream)))


def adam_groups(params: Gaussians, grads: Gaussians, m: Gaussians, v: Gaussians, lrs: dict,
                opacity_reg: bool = False):
    arr = (L.GsParamGroup * 5)()
    for k, f in enumerate(Gaussians.FIELDS):
        p = getattr(params, f)
        arr[k] = L.GsParamGroup(p.data_ptr(), getattr(grads, f).data_ptr(),
                                getattr(m, f).data_ptr(), getattr(v, f).data_ptr(), p.numel(),
                                float(lrs[f]), 1 if (opacity_reg and f == "opacity_logits") else 0)
    return arr


def adam_step(groups, step: int, beta1=0.9, beta2=0.999, eps=1e-15, lambda_o=0.0,
              reg_count=0, step_dev: Optional[torch.Tensor] = None, stream=None):
    L.check(L.lib().gs_adam_step(groups, len(groups), int(step), beta1, beta2, eps, lambda_o,
                                 int(reg_count), _ptr(step_dev), _stream(stream)))


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, stream=None):
    """Stable in-place LSD radix sort of uint64 keys (int64 tensor) and uint32
    values (int32 tensor) on the low key_bits bits."""
    if keys.dtype != torch.int64 or vals.dtype != torch.int32 or keys.numel() != vals.numel():
        raise ValueError("keys must be int64 and vals int32 of equal length")
    n = keys.numel()
    tmp = torch.empty(max(int(L.lib().gs_sort_tmp_bytes(n)), 256), dtype=torch.uint8,
                      device=keys.device)
    L.check(L.lib().gs_sort_pairs(_ptr(keys), _ptr(vals), n, int(key_bits), _ptr(tmp),
                                  _stream(stream)))


SORT_NOALLOC_MAX = 1 << 20


def sort_pairs_noalloc(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, stream=None):
    """sort_pairs without any allocation: the library's own per-GPU scratch
    (at most SORT_NOALLOC_MAX pairs; overlapping calls on one GPU race)."""
    if keys.dtype != torch.int64 or vals.dtype != torch.int32 or keys.numel() != vals.numel():
        raise ValueError("keys must be int64 and vals int32 of equal length")
    L.check(L.lib().gs_sort_pairs_noalloc(_ptr(keys), _ptr(vals), keys.numel(), int(key_bits),
                                          _stream(stream)))


def grad_stats(plan: Plan, ws: torch.Tensor, accum: torch.Tensor, denom: torch.Tensor,
               stream=None):
    """Accumulate the densification statistics of the last backward."""
    _check_ws(plan, ws)
    for t, name in ((accum, "accum"), (denom, "denom")):
        _need(t, name)
        if t.numel() != plan.n:
            raise ValueError(f"{name} must hold n floats")
    L.check(L.lib().gs_grad_stats(ctypes.byref(plan.c), _ptr(ws), _ptr(accum), _ptr(denom),
                                  _stream(stream)))


def densify_prune(g: Gaussians, m: Gaussians, v: Gaussians, accum: torch.Tensor,
                  denom: torch.Tensor, normals: torch.Tensor, tau_p: float = 0.001,
                  eps_alpha: float = 0.02, percent_dense: float = 0.01, extent: float = 1.0,
                  capacity: Optional[int] = None, stream=None):
    """Clone / split / prune; returns (params, m, v) with the new count
    (one host synchronisation to read it)."""
    n = g.n
    cap = 2 * n if capacity is None else int(capacity)
    if normals.numel() != 6 * n or accum.numel() != n or denom.numel() != n:
        raise ValueError("accum, denom must hold n floats and normals n x 2 x 3")
    mk = lambda: Gaussians(*[torch.empty((cap,) + tuple(x.shape[1:]), dtype=torch.float32,
                                         device=x.device) for x in g.tensors()], g.sh_degree)
    out, om, ov = mk(), mk(), mk()
    n_out = torch.zeros(1, dtype=torch.int32, device=g.means.device)
    tmp = torch.empty(max(int(L.lib().gs_densify_tmp_bytes(n)), 256), dtype=torch.uint8,
                      device=g.means.device)
    gc, mc, vc = g.c(), m.grads_c(), v.grads_c()
    oc, omc, ovc = out.grads_c(), om.grads_c(), ov.grads_c()
    L.check(L.lib().gs_densify_prune(ctypes.byref(gc), ctypes.byref(mc), ctypes.byref(vc),
                                     _ptr(accum), _ptr(denom), _ptr(normals), tau_p, eps_alpha,
                                     percent_dense, extent, ctypes.byref(oc), ctypes.byref(omc),
                                     ctypes.byref(ovc), cap, _ptr(n_out), _ptr(tmp),
                                     _stream(stream)))
    k = int(n_out.item())
    if k > cap:
        raise RuntimeError(f"densification needs {k} Gaussians, capacity {cap}")
    cut = lambda G: Gaussians(*[x[:k].contiguous() for x in G.tensors()], g.sh_degree)
    return cut(out), cut(om), cut(ov)


# ---------------------------------------------------------------- iterations

class Iteration:
    """All buffers of one mapping iteration over the plan's views, runnable
    eagerly (enqueue) or as a captured HIP graph (capture + replay)."""

    def __init__(self, plan: Plan, g: Gaussians, cams: torch.Tensor, target_rgb=None,
                 target_depth=None, dL_dcolor=None, dL_ddepth=None, pose_grad=False,
                 adam_lrs: Optional[dict] = None, lambda_o: float = 0.0, lambda_ssim: float = 0.0,
                 device="cuda", gather: Optional["KeyframePool"] = None,
                 adam_state: Optional[Tuple["Gaussians", "Gaussians", torch.Tensor]] = None):
        self.plan, self.g, self.cams = plan, g, cams
        _check_cams(plan, cams)
        if g.n != plan.n or g.sh_degree != plan.sh_degree:
            raise ValueError("Gaussians do not match the plan")
        P = plan.total_pixels
        for t, n, name in ((dL_dcolor, 3 * P, "dL_dcolor"), (dL_ddepth, P, "dL_ddepth"),
                           (target_rgb, 3 * P, "target_rgb"), (target_depth, P, "target_depth")):
            _check_img(t, n, name)
        self.ws = plan.new_workspace(device)
        self.frame = Frame(plan, device)
        self.grads = g.zeros_like()
        self.target_rgb, self.target_depth = target_rgb, target_depth
        self.dL_dcolor, self.dL_ddepth = dL_dcolor, dL_ddepth
        self.dL_dpose = (torch.zeros(plan.n_views, 6, dtype=torch.float32, device=device)
                         if pose_grad else None)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=device)
        self._graph = None
        self._groups = None
        if adam_lrs is not None:
            if adam_state is not None:
                # moments and step counter carried over (e.g. across a re-plan)
                self.m, self.v, self.step_dev = adam_state
            else:
                self.m, self.v = g.zeros_like(), g.zeros_like()
            self._groups = adam_groups(g, self.grads, self.m, self.v, adam_lrs, lambda_o != 0.0)
        it = L.GsIteration()
        it.plan = ctypes.pointer(plan.c)
        it.ws = self.ws.data_ptr()
        it.gaussians = g.c()
        it.cams_dev = cams.data_ptr()
        fr = self.frame
        it.color, it.depth, it.T_final, it.last = (fr.color.data_ptr(), fr.depth.data_ptr(),
                                                   fr.T_final.data_ptr(), fr.last.data_ptr())
        it.target_rgb = None if target_rgb is None else target_rgb.data_ptr()
        it.target_depth = None if target_depth is None else target_depth.data_ptr()
        it.loss_per_view = fr.loss.data_ptr() if target_rgb is not None else None
        it.dL_dcolor = None if dL_dcolor is None else dL_dcolor.data_ptr()
        it.dL_ddepth = None if dL_ddepth is None else dL_ddepth.data_ptr()
        it.grads = self.grads.grads_c()
        it.dL_dpose = None if self.dL_dpose is None else self.dL_dpose.data_ptr()
        if self._groups is not None:
            it.adam_groups = ctypes.cast(self._groups, ctypes.POINTER(L.GsParamGroup))
            it.n_adam_groups = len(self._groups)
        it.step_dev = self.step_dev.data_ptr()
        it.beta1, it.beta2, it.eps, it.lambda_o = 0.9, 0.999, 1e-15, float(lambda_o)
        it.reg_count = g.n
        self.loss_grad_color = self.loss_grad_depth = None
        if lambda_ssim > 0.0:
            self.loss_grad_color = torch.empty(3 * P, dtype=torch.float32, device=device)
            self.loss_grad_depth = torch.empty(P, dtype=torch.float32, device=device)
            it.lambda_ssim = float(lambda_ssim)
            it.loss_grad_color = self.loss_grad_color.data_ptr()
            it.loss_grad_depth = self.loss_grad_depth.data_ptr()
        self.gather = gather
        if gather is not None:
            # the iteration copies the keyframes of gather.sel into cams and
            # the targets first (they must be this iteration's own buffers)
            if target_rgb is None:
                raise ValueError("a gathered iteration needs target_rgb slots")
            if (gather.depth is None) != (target_depth is None):
                raise ValueError("the pool and the iteration must both have depth targets or neither")
            it.gather = ctypes.pointer(gather.c())
        self.c = it

    def enqueue(self, stream=None):
        L.check(L.lib().gs_iteration_enqueue(ctypes.byref(self.c), _stream(stream)))

    def capture(self, stream: torch.cuda.Stream):
        h = ctypes.c_void_p()
        L.check(L.lib().gs_graph_create(ctypes.byref(self.c), _stream(stream), ctypes.byref(h)))
        self._graph = h

    def replay(self, stream=None):
        L.check(L.lib().gs_graph_launch(self._graph, _stream(stream)))

    def time_graph(self, stream: torch.cuda.Stream, warmup: int = 3, reps: int = 20) -> float:
        """Mean ms per replay of the captured graph (HIP events, synchronises)."""
        ms = ctypes.c_float()
        L.check(L.lib().gs_graph_time(self._graph, _stream(stream), int(warmup), int(reps),
                                      ctypes.byref(ms)))
        return float(ms.value)

    MARKS = ["preprocess", "bin_scan", "bin_scatter", "bin_short_sort", "bin_long_sort",
             "forward", "loss", "raster_bwd", "project_bwd", "adam"]

    def time_marks(self, stream=None, warmup: int = 2, reps: int = 10):
        """Milliseconds of each launch group of an eagerly enqueued iteration
        (gs_iteration_time_marks: HIP events on the launch stream), as a
        [reps, len(MARKS)] float64 array; synchronises."""
        import numpy as np
        n = len(self.MARKS)
        buf = (ctypes.c_float * (reps * n))()
        L.check(L.lib().gs_iteration_time_marks(ctypes.byref(self.c), _stream(stream),
                                                int(warmup), int(reps), buf))
        return np.frombuffer(buf, dtype=np.float32).astype(np.float64).reshape(reps, n)

    def close(self):
        if self._graph is not None:
            L.check(L.lib().gs_graph_destroy(self._graph))
            self._graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- autograd

def spatial_order(means: torch.Tensor, stream=None) -> torch.Tensor:
    """Permutation (int32 [n], device) sorting the pool by the Morton code of
    its means (gs_spatial_order)."""
    _need(means, "means")
    n = means.shape[0]
    perm = torch.empty(n, dtype=torch.int32, device=means.device)
    tmp = torch.empty(max(int(L.lib().gs_spatial_order_tmp_bytes(n)), 256), dtype=torch.uint8,
                      device=means.device)
    L.check(L.lib().gs_spatial_order(_ptr(means), n, _ptr(perm), _ptr(tmp), _stream(stream)))
    return perm


def permute(g: "Gaussians", perm: torch.Tensor, stream=None) -> "Gaussians":
    """New Gaussians with row j = g's row perm[j] (gs_permute_gaussians)."""
    out = Gaussians(*[torch.empty_like(x) for x in g.tensors()], g.sh_degree)
    gc, oc = g.c(), out.grads_c()
    L.check(L.lib().gs_permute_gaussians(ctypes.byref(gc), _ptr(perm), ctypes.byref(oc),
                                         _stream(stream)))
    return out


spatial_order_ = spatial_order


class Mapper:
    """The mapping loop over one batch of views (Sec. IV-A): every iteration
    is one replay of the captured whole-iteration graph followed by the
    densification statistics; every `densify_every` iterations the pool is
    cloned / split / pruned (tau_p, eps_alpha), the moments follow their
    Gaussians, and the plan is rebuilt for the new count and captured again
    (the pair capacity with 30 % headroom over the new pool's pairs).  The
    split directions are drawn on the device from a seeded generator.  With
    spatial_order the pool (and the moments with it) is kept sorted by the
    Morton code of the means: re-ordered at the start and at every re-plan."""

    def __init__(self, g: Gaussians, cams: torch.Tensor, view_wh, target_rgb, target_depth,
                 lrs: dict, tile=(8, 8), lds_batch: int = 64, flags: int = 0,
                 densify_every: int = 500, tau_p: float = 0.001, eps_alpha: float = 0.02,
                 percent_dense: float = 0.01, extent: float = 1.0, seed: int = 0,
                 lambda_depth: float = 0.1, stream: Optional[torch.cuda.Stream] = None,
                 spatial_order: bool = False):
        self.cams, self.view_wh = cams, [tuple(v) for v in view_wh]
        self.target_rgb, self.target_depth, self.lrs = target_rgb, target_depth, lrs
        self.tile, self.lds_batch = tuple(tile), int(lds_batch)
        self.flags = int(flags) | L.GS_FUSED_L1
        self.densify_every, self.tau_p, self.eps_alpha = int(densify_every), tau_p, eps_alpha
        self.percent_dense, self.extent, self.lambda_depth = percent_dense, extent, lambda_depth
        self.gen = torch.Generator(device=g.means.device)
        self.gen.manual_seed(int(seed))
        self.stream = stream if stream is not None else torch.cuda.Stream(device=g.means.device)
        self.iterations, self.replans = 0, 0
        self.spatial_order = bool(spatial_order)
        if self.spatial_order:
            with torch.cuda.stream(self.stream):
                g = permute(g, spatial_order_(g.means, self.stream), self.stream)
            self.stream.synchronize()
        self._build(g, None)

    def _build(self, g: Gaussians, adam_state):
        dev = g.means.device
        cap = int(required_pairs(*g.tensors(), self.cams, self.view_wh, g.sh_degree, self.tile)
                  * 1.3) + 4096
        self.plan = Plan(g.n, g.sh_degree, self.view_wh, tile=self.tile,
                         lds_batch=self.lds_batch, flags=self.flags, pair_capacity=cap,
                         lambda_depth=self.lambda_depth)
        self.it = Iteration(self.plan, g, self.cams, target_rgb=self.target_rgb,
                            target_depth=self.target_depth, adam_lrs=self.lrs,
                            adam_state=adam_state)
        self.accum = torch.zeros(g.n, dtype=torch.float32, device=dev)
        self.denom = torch.zeros(g.n, dtype=torch.float32, device=dev)
        with torch.cuda.stream(self.stream):
            self.it.capture(self.stream)

    @property
    def g(self) -> Gaussians:
        return self.it.g

    def step(self):
        """One mapping iteration (and a densification when it is due)."""
        with torch.cuda.stream(self.stream):
            self.it.replay(self.stream)
            grad_stats(self.plan, self.it.ws, self.accum, self.denom, self.stream)
        self.iterations += 1
        if self.densify_every > 0 and self.iterations % self.densify_every == 0:
            self.densify()

    def densify(self):
        it = self.it
        with torch.cuda.stream(self.stream):
            normals = torch.randn(it.g.n, 2, 3, generator=self.gen, device=it.g.means.device)
            g, m, v = densify_prune(it.g, it.m, it.v, self.accum, self.denom, normals,
                                    tau_p=self.tau_p, eps_alpha=self.eps_alpha,
                                    percent_dense=self.percent_dense, extent=self.extent,
                                    stream=self.stream)
            if self.spatial_order:
                perm = spatial_order_(g.means, self.stream)
                g, m, v = (permute(x, perm, self.stream) for x in (g, m, v))
        self.stream.synchronize()
        step_dev = it.step_dev
        it.close()
        self._build(g, (m, v, step_dev))
        self.replans += 1

    def close(self):
        self.it.close()


class KeyframePool:
    """Keyframes of one camera size on the device -- camera records [K, 20],
    target colour [K, 3*H*W], target depth [K, H*W] (optional) -- and the
    batch selection `sel` [B] (int32, device) that a gathered Iteration
    renders: set it with select(ids) before each replay (an asynchronous
    copy on the stream)."""

    def __init__(self, cams: torch.Tensor, rgb: torch.Tensor, depth: Optional[torch.Tensor],
                 batch: int):
        _need(cams, "cams")
        _need(rgb, "rgb")
        if depth is not None:
            _need(depth, "depth")
        self.cams, self.rgb, self.depth = cams, rgb, depth
        self.n = cams.numel() // L.GS_CAMERA_FLOATS
        self.sel = torch.zeros(int(batch), dtype=torch.int32, device=cams.device)
        self._host = torch.zeros(int(batch), dtype=torch.int32).pin_memory()

    def c(self) -> "L.GsViewGather":
        g = L.GsViewGather()
        g.pool_cams, g.pool_rgb = self.cams.data_ptr(), self.rgb.data_ptr()
        g.pool_depth = None if self.depth is None else self.depth.data_ptr()
        g.sel, g.n_pool = self.sel.data_ptr(), self.n
        self._c = g
        return g

    def select(self, ids: Sequence[int], stream=None):
        if len(ids) != self.sel.numel() or not all(0 <= int(i) < self.n for i in ids):
            raise ValueError(f"need {self.sel.numel()} keyframe ids in [0, {self.n})")
        s = stream if stream is not None else torch.cuda.current_stream()
        s.synchronize()  # the pinned staging buffer is reused
        self._host.copy_(torch.tensor([int(i) for i in ids], dtype=torch.int32))
        with torch.cuda.stream(s):
            self.sel.copy_(self._host, non_blocking=True)


def pose_retract(cams: torch.Tensor, xi: torch.Tensor, out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Cameras at the poses R' = Exp(phi) R, t' = Exp(phi) t + rho for
    xi = [V, 6] (rho, phi) (gs_pose_retract)."""
    V = cams.numel() // L.GS_CAMERA_FLOATS
    _need(cams, "cams")
    _need(xi, "pose_tangent")
    if xi.numel() != 6 * V:
        raise ValueError("pose_tangent must hold n_views x 6 floats")
    out = torch.empty_like(cams) if out is None else out
    L.check(L.lib().gs_pose_retract(_ptr(cams), _ptr(xi), _ptr(out), V, _stream(stream)))
    return out


def pose_tangent_vjp(xi: torch.Tensor, g_delta: torch.Tensor, out: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    """dL/dxi from the camera gradient at the retracted pose (gs_pose_tangent_vjp)."""
    _need(xi, "pose_tangent")
    _need(g_delta, "dL_ddelta")
    V = xi.numel() // 6
    out = torch.empty_like(g_delta) if out is None else out
    L.check(L.lib().gs_pose_tangent_vjp(_ptr(xi), _ptr(g_delta), _ptr(out), V, _stream(stream)))
    return out


class Rasterizer:
    """Differentiable render of a fixed set of views (sizes, SH degree, tile
    configuration), reusable across calls: the plan is kept while the
    Gaussian count stays the same, and workspaces are pooled -- a forward
    takes one (allocating a zero-filled one only when none is free) and its
    backward returns it, so steady-state calls allocate nothing beyond
    torch's caching allocator.

    The pair capacity grows on demand: each forward reads the device flags
    once (one host synchronisation, the overflow check) and, if the pairs
    did not fit, re-plans with 25 % headroom and renders again.  With
    check_overflow=False there is no synchronisation; the caller then reads
    ``overflowed()`` after its own synchronisation.
    """

    def __init__(self, view_wh: Sequence[Tuple[int, int]], sh_degree: int, tile=_DEFAULT_TILE,
                 lds_batch: int = 256, flags: int = 0, pair_capacity: int = 1 << 16,
                 check_overflow: bool = True):
        self.view_wh = [(int(w), int(h)) for (w, h) in view_wh]
        self.sh_degree = int(sh_degree)
        self.tile, self.lds_batch = tuple(tile), int(lds_batch)
        self.flags = int(flags) & ~(L.GS_FUSED_L1 | L.GS_ACCUMULATE_GRADS)
        self.capacity = max(1, int(pair_capacity))
        self.check_overflow = check_overflow
        self.plan: Optional[Plan] = None
        self._free: List[torch.Tensor] = []
        self._last_ws: Optional[torch.Tensor] = None

    @property
    def n_views(self):
        return len(self.view_wh)

    def _plan_for(self, n: int) -> Plan:
        if self.plan is None or self.plan.n != n or self.plan.pair_capacity != self.capacity:
            self.plan = Plan(n, self.sh_degree, self.view_wh, tile=self.tile,
                             lds_batch=self.lds_batch, flags=self.flags,
                             pair_capacity=self.capacity)
            self._free = []   # workspaces of another layout
        return self.plan

    def acquire(self, device) -> torch.Tensor:
        plan = self.plan
        while self._free:
            ws = self._free.pop()
            if ws.numel() >= plan.ws_bytes and ws.device == torch.device(device):
                return ws
        return plan.new_workspace(device)

    def release(self, plan: Plan, ws: torch.Tensor):
        if plan is self.plan:
            self._free.append(ws)

    def overflowed(self) -> bool:
        """Whether the last forward's pairs exceeded the capacity (reads the
        device flags: synchronises)."""
        if self._last_ws is None:
            return False
        return bool(self.plan.flags_of(self._last_ws)[L.F_OVERFLOW])

    def forward_buffers(self, g: "Gaussians", cams: torch.Tensor):
        """Preprocess, binning and forward into fresh output buffers; returns
        (plan, ws, frame).  Retries once with a larger capacity on overflow."""
        for attempt in range(2):
            plan = self._plan_for(g.n)
            ws = self.acquire(g.means.device)
            preprocess(plan, ws, g, cams)
            bin_sort(plan, ws)
            fr = Frame(plan, g.means.device)
            render_fwd(plan, ws, cams, fr)
            self._last_ws = ws
            if not self.check_overflow:
                return plan, ws, fr
            fl = plan.flags_of(ws)
            if not fl[L.F_OVERFLOW]:
                return plan, ws, fr
            self.release(plan, ws)
            self.capacity = int(fl[L.F_PAIRS_WANTED] * 1.25) + 1024
            if self.capacity > 0x7FFFFFFF:
                break
        raise RuntimeError(f"pair capacity exceeded ({int(fl[L.F_PAIRS_WANTED])} pairs needed)")

    def __call__(self, means, log_scales, quats, opacity_logits, sh, cams: torch.Tensor,
                 pose_tangent: Optional[torch.Tensor] = None):
        # a backward will come only when autograd records this call; otherwise
        # the forward hands its workspace back to the pool at once
        keep = torch.is_grad_enabled() and any(
            t is not None and t.requires_grad
            for t in (means, log_scales, quats, opacity_logits, sh, pose_tangent))
        return _Rasterize.apply(means, log_scales, quats, opacity_logits, sh, pose_tangent,
                                cams, self, keep)


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, pose_tangent, cams, rz, keep):
        g = Gaussians(means.detach().contiguous(), log_scales.detach().contiguous(),
                      quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                      sh.detach().contiguous(), rz.sh_degree)
        _need(cams, "cams")
        xi = None
        if pose_tangent is not None:
            xi = pose_tangent.detach().contiguous()
            cams = pose_retract(cams, xi)
        plan, ws, fr = rz.forward_buffers(g, cams)
        if keep:
            ctx.rz, ctx.plan, ctx.ws, ctx.frame, ctx.g, ctx.cams, ctx.xi = (
                rz, plan, ws, fr, g, cams, xi)
        else:
            rz.release(plan, ws)
        ctx.mark_non_differentiable(fr.T_final)
        return fr.color, fr.depth, fr.T_final

    @staticmethod
    def backward(ctx, g_color, g_depth, g_T):
        plan, g = ctx.plan, ctx.g
        dev = g.means.device
        grads = Gaussians(*[torch.empty_like(x) for x in g.tensors()], g.sh_degree)
        want_pose = ctx.xi is not None and ctx.needs_input_grad[5]
        dpose = torch.empty(plan.n_views, 6, dtype=torch.float32, device=dev) if want_pose else None
        gc = torch.zeros_like(ctx.frame.color) if g_color is None else g_color.contiguous()
        gd = None if g_depth is None else g_depth.contiguous()
        render_bwd(plan, ctx.ws, g, ctx.cams, ctx.frame, grads, dL_dcolor=gc, dL_ddepth=gd,
                   dL_dpose=dpose)
        ctx.rz.release(plan, ctx.ws)
        ctx.ws = None
        dxi = pose_tangent_vjp(ctx.xi, dpose) if want_pose else None
        return (grads.means, grads.log_scales, grads.quats, grads.opacity_logits,
                grads.sh.view_as(g.sh), dxi, None, None, None)


_RASTERIZERS = {}


def rasterize(means, log_scales, quats, opacity_logits, sh, cams: torch.Tensor,
              view_wh: Sequence[Tuple[int, int]], sh_degree: int, pose_tangent=None,
              tile=_DEFAULT_TILE, lds_batch: int = 256, pair_capacity: Optional[int] = None):
    """Differentiable render of one or more views.

    Returns (color [3*P], depth [P], T_final [P]) concatenated over views
    (split with Plan.split_views).  Gradients flow to the five parameter
    tensors and to ``pose_tangent`` ([V, 6] = (rho, phi)): the views are
    rendered at R' = Exp(phi) R, t' = Exp(phi) t + rho (gs_pose_retract),
    and dL/dxi is the camera gradient pulled back through that map
    (gs_pose_tangent_vjp; at xi = 0 it is the camera gradient itself).
    Plans and workspaces are cached per (view sizes, degree, tile, LDS
    batch); the pair capacity grows on demand (see Rasterizer).
    """
    key = (tuple((int(w), int(h)) for (w, h) in view_wh), int(sh_degree), tuple(tile),
           int(lds_batch), str(means.device))
    rz = _RASTERIZERS.get(key)
    if rz is None:
        rz = Rasterizer(view_wh, sh_degree, tile=tile, lds_batch=lds_batch)
        _RASTERIZERS[key] = rz
    if pair_capacity is not None and int(pair_capacity) > rz.capacity:
        rz.capacity = int(pair_capacity)
    return rz(means, log_scales, quats, opacity_logits, sh, cams, pose_tangent)


def required_pairs(means, log_scales, quats, opacity_logits, sh, cams, view_wh, sh_degree,
                   tile=_DEFAULT_TILE) -> int:
    """Exact (Gaussian, tile) pair count of the current parameters."""
    plan = Plan(int(means.shape[0]), sh_degree, view_wh, tile=tile, pair_capacity=1)
    ws = plan.new_workspace(means.device)
    g = Gaussians(means.detach().contiguous(), log_scales.detach().contiguous(),
                  quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                  sh.detach().contiguous(), sh_degree)
    preprocess(plan, ws, g, cams)
    bin_sort(plan, ws)
    return int(plan.flags_of(ws)[L.F_PAIRS_WANTED])
