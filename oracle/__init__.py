"""FP64 CPU oracle of the differentiable 3DGS rasterizer -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and never falls back to it.

The arithmetic lives in ``oracle.cpp`` (double precision, plain loops,
OpenMP over pixels / tiles / Gaussians); this module marshals numpy arrays
and adds the pieces that are library routines or one-line definitions:

* the L1 photometric loss of Eq. (9) (its L1 part, with the depth term of the
  RGB-D workloads) and its gradient with sign(0) = 0;
* the Adam step with torch.optim.Adam semantics (the optimiser 3DGS uses,
  which the paper retains, Sec. IV-A);
* the opacity regulariser of Eq. (10), L_o = mean(|sigmoid(logit)|);
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_I64 = ctypes.c_int64
_I = ctypes.c_int


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "oracle.cpp"))):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.ora_preprocess.argtypes = [_I64, _I, _dp, _dp, _dp, _dp, _dp, _dp, _I, _I, _I, _I, _I,
                                     _dp, _dp, _dp, _dp, _dp, _dp, _fp, _i32, _i32, _u8, _i32, _i32]
        L.ora_preprocess.restype = None
        L.ora_sort_pairs.argtypes = [_I64, _i32, _i32, _fp, _I, _I, _u64, _u32, _u32]
        L.ora_sort_pairs.restype = _I64
        L.ora_render_fwd.argtypes = [_I, _I, _I, _I, _dp, _dp, _dp, _dp, _dp, _u32, _u32, _dp,
                                     _dp, _dp, _dp, _i32, _i32, _I]
        L.ora_render_fwd.restype = None
        L.ora_flag_decisions.argtypes = [_I, _I, _I, _I, _dp, _dp, _dp, _dp, _dp, _u32, _u32,
                                         _dp, _I64, _i32, _i32, _i32]
        L.ora_flag_decisions.restype = _I64
        L.ora_render_untiled.argtypes = [_I, _I, _I64, _i32, _dp, _dp, _dp, _dp, _dp, _fp, _dp,
                                         _dp, _dp, _dp, _i32]
        L.ora_render_untiled.restype = None
        L.ora_render_bwd.argtypes = [_I, _I, _I, _I, _I64, _I64, _dp, _dp, _dp, _dp, _dp, _u32,
                                     _u32, _dp, _dp, ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp,
                                     _I]
        L.ora_render_bwd.restype = None
        L.ora_project_bwd.argtypes = [_I64, _I, _dp, _dp, _dp, _dp, _dp, _dp, _I, _I, _I, _I, _I,
                                      _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.ora_project_bwd.restype = None
        L.ora_covariance3d.argtypes = [_I64, _dp, _dp, _dp]
        L.ora_covariance3d.restype = None
        _lib = L
    return _lib


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cam64(cam):
    """Camera record (fx fy cx cy R[9] t[3] near bg[3]) in float64; the
    camera's own arrays are used at whatever precision they hold."""
    return np.concatenate([
        np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float64),
        np.asarray(cam.R, np.float64).reshape(9), np.asarray(cam.t, np.float64).reshape(3),
        np.array([cam.near], np.float64), np.asarray(cam.bg, np.float64)])


def covariance3d(log_scales, quats):
    """World covariance R(q) diag(exp(2 l)) R^T per Gaussian, [n,3,3]."""
    ls = _c64(log_scales).reshape(-1, 3)
    q = _c64(quats).reshape(-1, 4)
    out = np.zeros((ls.shape[0], 9))
    lib().ora_covariance3d(ls.shape[0], ls, q, out)
    return out.reshape(-1, 3, 3)


def _tiles(cam, tile):
    tw, th = tile
    return (cam.width + tw - 1) // tw, (cam.height + th - 1) // th


def preprocess(scene, cam, tile=(16, 16), cutoff="exact") -> Dict[str, np.ndarray]:
    """Per-Gaussian projection of ``scene`` into ``cam`` (FP64)."""
    n = scene.n
    out = dict(
        mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), cov2d=np.zeros((n, 3)),
        opacity=np.zeros(n), rgb=np.zeros((n, 3)), depth=np.zeros(n),
        depth32=np.zeros(n, np.float32), rect=np.zeros((n, 4), np.int32),
        tiles_touched=np.zeros(n, np.int32), clamp_mask=np.zeros(n, np.uint8),
        status=np.zeros(n, np.int32), near_edge=np.zeros(n, np.int32))
    lib().ora_preprocess(
        n, scene.sh_degree, _c64(scene.means), _c64(scene.log_scales), _c64(scene.quats),
        _c64(scene.opacity_logits), _c64(scene.sh), _cam64(cam), cam.width, cam.height,
        tile[0], tile[1], 1 if cutoff == "3sigma" else 0,
        out["mean2d"], out["conic"], out["cov2d"], out["opacity"], out["rgb"], out["depth"],
        out["depth32"], out["rect"], out["tiles_touched"], out["clamp_mask"], out["status"],
        out["near_edge"])
    return out


def sort_pairs(pre, cam, tile=(16, 16)):
    """Stable sort of the (tile, float32-depth) keys; returns keys, vals, ranges."""
    tx, ty = _tiles(cam, tile)
    P = int(pre["tiles_touched"].astype(np.int64).sum())
    keys = np.zeros(max(P, 1), np.uint64)
    vals = np.zeros(max(P, 1), np.uint32)
    ranges = np.zeros(2 * tx * ty, np.uint32)
    P2 = lib().ora_sort_pairs(pre["status"].shape[0], pre["rect"], pre["tiles_touched"],
                              pre["depth32"], tx, tx * ty, keys, vals, ranges)
    assert P2 == P
    return keys[:P], vals[:P], ranges


def render(scene, cam, tile=(16, 16), cutoff="exact", pre=None, flip_band=False):
    """Tiled forward render of one view.  Returns a dict with color [3,H,W],
    depth, T_final, last, flag (pixels near a discrete decision), and the
    preprocess / sort products.  flip_band: every decision within a relative
    1e-5 of its threshold takes the other branch (for the tests' sensitivity
    of a result to those decisions)."""
    if pre is None:
        pre = preprocess(scene, cam, tile, cutoff)
    keys, vals, ranges = sort_pairs(pre, cam, tile)
    H, W = cam.height, cam.width
    color = np.zeros((3, H, W)); depth = np.zeros((H, W)); T = np.zeros((H, W))
    last = np.zeros((H, W), np.int32); flag = np.zeros((H, W), np.int32)
    lib().ora_render_fwd(W, H, tile[0], tile[1], pre["mean2d"], pre["conic"], pre["opacity"],
                         pre["rgb"], pre["depth"], np.ascontiguousarray(vals), ranges,
                         _c64(cam.bg), color, depth, T, last, flag, 1 if flip_band else 0)
    return dict(color=color, depth=depth, T_final=T, last=last, flag=flag, pre=pre,
                keys=keys, vals=vals, ranges=ranges, flip_band=flip_band)


def flag_decisions(fwd, cam, tile=(16, 16)):
    """Decisions of ``fwd`` (a result of render) taken within a relative 1e-5
    of their thresholds.  Returns int arrays (pixel, gaussian, kind): kind 1
    the 0.99 clamp, 2 the 1/255 skip, 4 the 1e-4 stop (the Gaussian whose
    decision it is), 8 a Gaussian blended at a pixel that has such a
    decision."""
    pre = fwd["pre"]
    args = (cam.width, cam.height, tile[0], tile[1], pre["mean2d"], pre["conic"],
            pre["opacity"], pre["rgb"], pre["depth"], np.ascontiguousarray(fwd["vals"]),
            fwd["ranges"], _c64(cam.bg))
    cap = 1 << 16
    while True:
        pix, g, kind = (np.zeros(cap, np.int32) for _ in range(3))
        total = lib().ora_flag_decisions(*args, cap, pix, g, kind)
        if total <= cap:
            return pix[:total], g[:total], kind[:total]
        cap = int(total)


def render_untiled(scene, cam, pre=None):
    """Brute force: every visible Gaussian for every pixel (small scenes)."""
    if pre is None:
        pre = preprocess(scene, cam)
    H, W = cam.height, cam.width
    color = np.zeros((3, H, W)); depth = np.zeros((H, W)); T = np.zeros((H, W))
    nb = np.zeros((H, W), np.int32)
    lib().ora_render_untiled(W, H, scene.n, pre["status"], pre["mean2d"], pre["conic"],
                             pre["opacity"], pre["rgb"], pre["depth"], pre["depth32"],
                             _c64(cam.bg), color, depth, T, nb)
    return dict(color=color, depth=depth, T_final=T, n_blended=nb)


def backward_2d(scene, cam, dL_dcolor, dL_ddepth=None, tile=(16, 16), cutoff="exact", fwd=None,
                flip_band=False):
    """Per-Gaussian 2D gradients of one view (mean2d, conic, opacity, rgb, depth).
    flip_band as in render (taken from ``fwd`` when given)."""
    if fwd is None:
        fwd = render(scene, cam, tile, cutoff, flip_band=flip_band)
    flip_band = fwd.get("flip_band", False)
    pre = fwd["pre"]
    n = scene.n
    H, W = cam.height, cam.width
    g = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n),
             rgb=np.zeros((n, 3)), depth=np.zeros(n))
    gd = None if dL_ddepth is None else _c64(dL_ddepth).reshape(H * W)
    lib().ora_render_bwd(W, H, tile[0], tile[1], n, int(fwd["vals"].shape[0]), pre["mean2d"],
                         pre["conic"], pre["opacity"], pre["rgb"], pre["depth"],
                         np.ascontiguousarray(fwd["vals"]), fwd["ranges"], _c64(cam.bg),
                         _c64(dL_dcolor).reshape(3 * H * W),
                         None if gd is None else gd.ctypes.data_as(ctypes.c_void_p),
                         g["mean2d"], g["conic"], g["opacity"], g["rgb"], g["depth"],
                         1 if flip_band else 0)
    if gd is not None:
        g["_keep"] = gd
    return g


def project_backward(scene, cam, g2d, tile=(16, 16), cutoff="exact", accum=None):
    """Chain rule to parameter gradients (added into ``accum`` if given) and
    the camera tangent gradient (rho, phi) of this view."""
    n = scene.n
    K = (scene.sh_degree + 1) ** 2
    if accum is None:
        accum = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)),
                     quats=np.zeros((n, 4)), opacity_logits=np.zeros(n),
                     sh=np.zeros((n, K, 3)))
    pose = np.zeros(6)
    lib().ora_project_bwd(
        n, scene.sh_degree, _c64(scene.means), _c64(scene.log_scales), _c64(scene.quats),
        _c64(scene.opacity_logits), _c64(scene.sh), _cam64(cam), cam.width,
        cam.height, tile[0], tile[1], 1 if cutoff == "3sigma" else 0,
        _c64(g2d["mean2d"]), _c64(g2d["conic"]), _c64(g2d["opacity"]), _c64(g2d["rgb"]),
        _c64(g2d["depth"]), accum["means"], accum["log_scales"], accum["quats"],
        accum["opacity_logits"], accum["sh"], pose)
    return accum, pose


def backward(scene, cams, dL_dcolor, dL_ddepth=None, tile=(16, 16), cutoff="exact",
             flip_band=False):
    """Full backward over one or more views: parameter gradients summed over
    views, and one camera-tangent gradient per view."""
    if not isinstance(cams, (list, tuple)):
        cams, dL_dcolor, dL_ddepth = [cams], [dL_dcolor], [dL_ddepth]
    if dL_ddepth is None:
        dL_ddepth = [None] * len(cams)
    accum, poses = None, []
    for cam, gc, gd in zip(cams, dL_dcolor, dL_ddepth):
        g2d = backward_2d(scene, cam, gc, gd, tile, cutoff, flip_band=flip_band)
        accum, pose = project_backward(scene, cam, g2d, tile, cutoff, accum)
        poses.append(pose)
    return accum, np.stack(poses)


def _hat(v):
    x, y, z = (float(a) for a in v)
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def so3_exp(phi):
    """Rotation matrix of the rotation vector phi (scipy's rotvec map)."""
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(np.asarray(phi, np.float64)).as_matrix()


def so3_left_jacobian(phi, terms=40):
    """Left Jacobian of SO(3) from its defining power series
    J(phi) = sum_k [phi]x^k / (k+1)!  (so that Exp(phi + d) = Exp(J d) Exp(phi)
    to first order in d)."""
    K = _hat(phi)
    J = np.zeros((3, 3))
    P = np.eye(3)
    fact = 1.0
    for k in range(terms):
        fact *= (k + 1)
        J += P / fact
        P = P @ K
    return J


def retract_camera(cam, xi, round32=True):
    """The camera at the pose R' = Exp(phi) R, t' = Exp(phi) t + rho, xi =
    (rho, phi): the left perturbation the camera gradient is taken for.
    round32: store R', t' as float32, the type of the device camera record."""
    import dataclasses
    xi = np.asarray(xi, np.float64)
    E = so3_exp(xi[3:6])
    R = E @ np.asarray(cam.R, np.float64)
    t = E @ np.asarray(cam.t, np.float64) + xi[0:3]
    if round32:
        R, t = R.astype(np.float32), t.astype(np.float32)
    return dataclasses.replace(cam, R=R, t=t)


def pose_tangent_vjp(xi, g_delta):
    """dL/dxi of L(retract(xi)) from g_delta = dL/ddelta, the gradient of a
    left perturbation at the retracted pose: with Exp(phi + dphi) =
    Exp(J dphi) Exp(phi), a step dxi is the perturbation delta = (drho +
    rho x (J dphi), J dphi), so dL/drho = g_rho, dL/dphi = J^T (g_phi - rho x
    g_rho)."""
    xi = np.asarray(xi, np.float64).reshape(-1, 6)
    g = np.asarray(g_delta, np.float64).reshape(-1, 6)
    out = np.zeros_like(g)
    for v in range(xi.shape[0]):
        rho, phi = xi[v, :3], xi[v, 3:]
        J = so3_left_jacobian(phi)
        out[v, :3] = g[v, :3]
        out[v, 3:] = J.T @ (g[v, 3:] - np.cross(rho, g[v, :3]))
    return out


def linear_loss(fwd_list, dL_dcolor, dL_ddepth=None):
    """L = sum(gC * C) + sum(gD * D) over views (for finite differences)."""
    total = 0.0
    for k, f in enumerate(fwd_list):
        total += float(np.sum(np.asarray(dL_dcolor[k], np.float64) * f["color"]))
        if dL_ddepth is not None and dL_ddepth[k] is not None:
            total += float(np.sum(np.asarray(dL_ddepth[k], np.float64) * f["depth"]))
    return total


def l1_loss_and_grads(color, depth, target_rgb, target_depth, lambda_depth):
    """L1 part of Eq. (9) with a depth term: mean |C - C*| over pixels and
    channels plus lambda_depth * mean |D - D*| over pixels.  sign(0) = 0."""
    npx = color.shape[1] * color.shape[2]
    d = np.asarray(color, np.float64) - np.asarray(target_rgb, np.float64)
    loss = np.abs(d).sum() / (3.0 * npx)
    gC = np.sign(d) / (3.0 * npx)
    gD = np.zeros(color.shape[1:])
    if target_depth is not None and lambda_depth != 0.0:
        dd = np.asarray(depth, np.float64) - np.asarray(target_depth, np.float64)
        loss += lambda_depth * np.abs(dd).sum() / npx
        gD = lambda_depth * np.sign(dd) / npx
    return loss, gC, gD


def opacity_reg_grad(logits, lambda_o, n_total=None):
    """Gradient of lambda_o * L_o, L_o = (1/N) sum_i |o_i|, o_i = sigmoid(logit_i)
    (Eq. (10)); the activated opacity is positive so |o| = o."""
    x = np.asarray(logits, np.float64)
    n = x.size if n_total is None else n_total
    o = 1.0 / (1.0 + np.exp(-x))
    return lambda_o * o * (1.0 - o) / n


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (torch.optim.Adam semantics, no weight decay), FP64,
    returning new (p, m, v)."""
    p = np.asarray(p, np.float64); g = np.asarray(g, np.float64)
    m = np.asarray(m, np.float64); v = np.asarray(v, np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    denom = np.sqrt(v) / np.sqrt(bc2) + eps
    p = p - (lr / bc1) * m / denom
    return p, m, v
