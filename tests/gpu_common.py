"""Shared helpers of the GPU parity tests (imported by tests/test_gpu_*.py)."""
import functools

import numpy as np
import torch

import oracle
import paper_2410_00486_amd as gsr
from paper_2410_00486_amd import _lib as L
from synth import scenes

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

# forward tolerance: |g - o| <= 1e-5 |o| + 1e-7 per element (colour, depth)
FWD_RTOL, FWD_ATOL = 1e-5, 1e-7
# gradients: |g - o| <= 1e-3 |o| + 1e-3 rms(o) per element, and a 1e-4
# relative error of the whole tensor
GRAD_RTOL, GRAD_ATOL_RMS, GRAD_NORM = 1e-3, 1e-3, 1e-4


@functools.lru_cache(maxsize=None)
def workload(cfg: int, **kw):
    return scenes.WORKLOADS[cfg](**kw)


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def run_gpu(scene, cams, tile=(16, 16), lds=256, flags=0, dL_dcolor=None, dL_ddepth=None,
            target_rgb=None, target_depth=None, pose=False, capacity=None, lambda_depth=0.1,
            chunk=2):
    g = gsr.Gaussians.from_scene(scene, DEV)
    ct = gsr.cameras_tensor(cams, DEV)
    wh = [(c.width, c.height) for c in cams]
    if capacity is None:
        capacity = gsr.required_pairs(*g.tensors(), ct, wh, scene.sh_degree, tile) + 7
    plan = gsr.Plan(scene.n, scene.sh_degree, wh, tile=tile, lds_batch=lds, flags=flags,
                    pair_capacity=max(1, capacity), lambda_depth=lambda_depth, chunk=chunk)
    flat = lambda xs: None if xs is None else t32(np.concatenate([np.asarray(x).reshape(-1) for x in xs]))
    if dL_dcolor is None and not (flags & L.GS_FUSED_L1):
        # forward-focused cases still run the whole iteration: zero upstream gradient
        dL_dcolor = [np.zeros((3, c.height, c.width), np.float32) for c in cams]
    it = gsr.Iteration(plan, g, ct, target_rgb=flat(target_rgb), target_depth=flat(target_depth),
                       dL_dcolor=flat(dL_dcolor), dL_ddepth=flat(dL_ddepth), pose_grad=pose)
    it.enqueue()
    torch.cuda.synchronize()
    return it


def view_images(it, v):
    plan = it.plan
    col = plan.split_views(it.frame.color, 3)[v].cpu().numpy().astype(np.float64)
    dep = plan.split_views(it.frame.depth)[v].cpu().numpy().astype(np.float64)
    T = plan.split_views(it.frame.T_final)[v].cpu().numpy().astype(np.float64)
    last = plan.split_views(it.frame.last)[v].cpu().numpy()
    return col, dep, T, last


def grads_np(it):
    return {f: getattr(it.grads, f).cpu().numpy().astype(np.float64) for f in gsr.Gaussians.FIELDS}


def flagged_gaussians(ref, tile, cam):
    """Gaussians whose tile box covers a tile holding a flagged pixel, or whose
    rect edge / depth rounding is itself flagged."""
    pre = ref["pre"]
    tx = (cam.width + tile[0] - 1) // tile[0]
    ty = (cam.height + tile[1] - 1) // tile[1]
    fl = np.zeros((ty * tile[1], tx * tile[0]), bool)
    fl[:cam.height, :cam.width] = ref["flag"] != 0
    tflag = fl.reshape(ty, tile[1], tx, tile[0]).any(axis=(1, 3))
    bad = pre["near_edge"] != 0
    for i in np.nonzero((pre["status"] == 1) & ~bad)[0]:
        x0, y0, x1, y1 = pre["rect"][i]
        if tflag[y0:y1, x0:x1].any():
            bad[i] = True
    return bad


def assert_forward_close(col, dep, ref, extra_mask=None, max_flag_frac=1e-4):
    ok = ref["flag"] == 0
    if extra_mask is not None:
        ok &= extra_mask
    n_flag = int((~ok).sum())
    assert n_flag <= max(10, max_flag_frac * ok.size), f"{n_flag} flagged pixels"
    for name, g, o in (("color", col[:, ok], ref["color"][:, ok]), ("depth", dep[ok], ref["depth"][ok])):
        err = np.abs(g - o)
        lim = FWD_RTOL * np.abs(o) + FWD_ATOL
        bad = err > lim
        assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} outside tolerance, "
                               f"worst excess {float((err / lim).max()):.3g}x")
    return n_flag


def assert_grads_close(got: dict, ref: dict, exclude=None, fields=gsr.Gaussians.FIELDS):
    report = {}
    for f in fields:
        g = got[f].reshape(got[f].shape[0], -1)
        o = ref[f].reshape(ref[f].shape[0], -1)
        if exclude is not None:
            g, o = g[~exclude], o[~exclude]
        rms = float(np.sqrt(np.mean(o * o))) if o.size else 0.0
        err = np.abs(g - o)
        lim = GRAD_RTOL * np.abs(o) + GRAD_ATOL_RMS * rms
        nrm = float(np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-300))
        report[f] = (float((err / np.maximum(lim, 1e-300)).max()) if o.size else 0.0, nrm)
        assert (err <= lim).all(), f"{f}: {int((err > lim).sum())} elements out of tolerance; {report[f]}"
        assert nrm <= GRAD_NORM, f"{f}: relative norm error {nrm:.3g}"
    return report
