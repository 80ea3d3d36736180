"""Adaptive densification and opacity pruning -- TEST INFRASTRUCTURE (FP64).

The paper densifies every 500 iterations with a positional-gradient
threshold tau_p = 0.001 and removes Gaussians with opacity below
eps_alpha = 0.02 (Sec. IV-A), by splitting and cloning as in 3DGS, whose
conventions it retains (Sec. III-A, adaptive densification):

* statistics: after each backward, every Gaussian visible in a view adds
  the norm of its screen-space mean gradient expressed in normalised device
  coordinates, |(g_x W/2, g_y H/2)| (g in pixel units), to `accum` and 1 to
  `denom`;
* a Gaussian is selected when denom > 0 and accum / denom >= tau_p;
* a selected Gaussian whose largest scale is <= percent_dense * extent is
  cloned (the original and an identical copy); a larger one is split into
  two children with means p + R(q) (s * n_k) (n_k standard normal draws,
  passed in), scales s / 1.6, the same rotation, opacity and colour;
* every Gaussian (original, copy or child) with sigmoid(logit) < eps_alpha
  is removed;
* these three decisions are taken in float32 (the library's precision);
* output order: Gaussians in input order, each followed by its copy, or
  replaced by its two children; Adam moments are kept for kept originals and
  zero for copies and children; the statistics restart at zero.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def accumulate_stats(accum, denom, g_mean2d, visible, width, height):
    """One view: accum += |(gx W/2, gy H/2)| for visible Gaussians."""
    g = np.asarray(g_mean2d, np.float64)
    norm = np.sqrt((g[:, 0] * width / 2.0) ** 2 + (g[:, 1] * height / 2.0) ** 2)
    vis = np.asarray(visible, bool)
    accum = np.asarray(accum, np.float64) + np.where(vis, norm, 0.0)
    denom = np.asarray(denom, np.float64) + vis.astype(np.float64)
    return accum, denom


def _rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def densify_prune(params: dict, m: dict, v: dict, accum, denom, normals, tau_p=0.001,
                  eps_alpha=0.02, percent_dense=0.01, extent=1.0):
    """Returns (params', m', v') as float32 dicts; normals is [n, 2, 3]."""
    n = params["means"].shape[0]
    out = {f: [] for f in FIELDS}
    om = {f: [] for f in FIELDS}
    ov = {f: [] for f in FIELDS}

    def emit(vals, mm, vv):
        for f in FIELDS:
            out[f].append(vals[f])
            om[f].append(mm[f])
            ov[f].append(vv[f])

    zero = lambda i: {f: np.zeros_like(np.asarray(params[f][i], np.float32)) for f in FIELDS}
    f32 = np.float32
    for i in range(n):
        # the discrete decisions are taken in float32, the library's precision
        logit = f32(params["opacity_logits"][i])
        if not (f32(1) / (f32(1) + np.exp(-logit)) >= f32(eps_alpha)):
            continue
        own = {f: np.asarray(params[f][i], np.float32) for f in FIELDS}
        own_m = {f: np.asarray(m[f][i], np.float32) for f in FIELDS}
        own_v = {f: np.asarray(v[f][i], np.float32) for f in FIELDS}
        sel = f32(denom[i]) > 0 and f32(accum[i]) / f32(denom[i]) >= f32(tau_p)
        if not sel:
            emit(own, own_m, own_v)
            continue
        s = np.exp(np.asarray(params["log_scales"][i], np.float64))
        smax32 = np.exp(f32(np.max(np.asarray(params["log_scales"][i], np.float32))))
        if smax32 <= f32(percent_dense) * f32(extent):
            emit(own, own_m, own_v)
            emit(own, zero(i), zero(i))
        else:
            R = _rot(params["quats"][i])
            for k in range(2):
                child = dict(own)
                p = np.asarray(params["means"][i], np.float64) + R @ (s * np.asarray(normals[i, k], np.float64))
                child["means"] = p.astype(np.float32)
                child["log_scales"] = (np.asarray(params["log_scales"][i], np.float64)
                                       - np.log(1.6)).astype(np.float32)
                emit(child, zero(i), zero(i))
    res = []
    for d in (out, om, ov):
        res.append({f: (np.stack(d[f]).astype(np.float32) if d[f] else
                        np.zeros((0,) + np.asarray(params[f]).shape[1:], np.float32)) for f in FIELDS})
    return tuple(res)
