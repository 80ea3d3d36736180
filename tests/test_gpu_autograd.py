"""The torch.autograd path (rasterize / Rasterizer) against the FP64 oracle:
forward colour and depth, the gradients of all five parameter tensors and of
the camera tangent (at zero and away from it), a directional FP32 finite
difference through the autograd function itself, and the on-demand growth
of the pair capacity.  Upstream gradients come from fixed linear losses
(no L1 kinks)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_00486_amd as gsr
from synth import scenes

from gpu_common import (DEV, assert_forward_close, assert_grads_close, assert_pose_close,
                        oracle_reference, t32, visible_count, workload)

pytestmark = pytest.mark.gpu

FIELDS = gsr.Gaussians.FIELDS


def _leaves(scene):
    g = gsr.Gaussians.from_scene(scene, DEV)
    return [x.clone().requires_grad_(True) for x in g.tensors()]


def _render(scene, cams, xi=None, tile=(16, 16)):
    leaves = _leaves(scene)
    ct = gsr.cameras_tensor(cams, DEV)
    wh = [(c.width, c.height) for c in cams]
    xt = None if xi is None else t32(xi).reshape(len(cams), 6).requires_grad_(True)
    col, dep, T = gsr.rasterize(*leaves, ct, wh, scene.sh_degree, pose_tangent=xt, tile=tile)
    return leaves, xt, col, dep, T


def _linear_backward(col, dep, gcs, gds):
    gc = t32(np.concatenate([g.reshape(-1) for g in gcs]))
    gd = t32(np.concatenate([g.reshape(-1) for g in gds]))
    loss = (col * gc).sum() + (dep * gd).sum()
    loss.backward()
    return loss


def _grads(leaves):
    return {f: x.grad.detach().cpu().numpy().astype(np.float64) for f, x in zip(FIELDS, leaves)}


@pytest.mark.parametrize("cfg", [1, 3])
def test_rasterize_matches_oracle(cfg):
    """Forward, the five parameter gradients and the camera tangent at zero."""
    w = workload(cfg)
    cam = w.cameras[0]
    print(f"autograd rasterize workload {cfg}", flush=True)
    leaves, xt, col, dep, T = _render(w.scene, [cam], xi=np.zeros(6))
    ref = oracle.render(w.scene, cam)
    H, W = cam.height, cam.width
    assert_forward_close(col.detach().view(3, H, W).cpu().numpy().astype(np.float64),
                         dep.detach().view(H, W).cpu().numpy().astype(np.float64), ref)
    gcs, gds = scenes.linear_loss_weights(300 + cfg, [cam])
    _linear_backward(col, dep, gcs, gds)
    torch.cuda.synchronize()
    grads, poses, exclude, poses_f = oracle_reference(w.scene, [cam], gcs, gds)
    assert_grads_close(_grads(leaves), grads, exclude, visible=visible_count(w.scene, [cam]))
    assert_pose_close(xt.grad.cpu().numpy(), poses, poses_f)


def test_rasterize_nonzero_pose_tangent_two_views():
    """Two views rendered at retracted poses R' = Exp(phi) R, t' = Exp(phi) t
    + rho: the images against the oracle at the same (float32) poses, the
    parameter gradients, and dL/dxi against the oracle's camera gradient at
    the retracted pose pulled back through the SO(3) left Jacobian."""
    w = workload(3)
    cams = [w.cameras[0], w.gt_cameras[0]]
    xi = np.array([[0.01, -0.02, 0.015, 0.02, -0.01, 0.03],
                   [-0.015, 0.01, 0.02, -0.03, 0.02, 0.01]])
    print("autograd rasterize, two views, nonzero tangent", flush=True)
    leaves, xt, col, dep, T = _render(w.scene, cams, xi=xi)
    rcams = [oracle.retract_camera(c, x) for c, x in zip(cams, xi)]
    H, W = cams[0].height, cams[0].width
    for v, rc in enumerate(rcams):
        ref = oracle.render(w.scene, rc)
        o = v * H * W
        c = col.detach()[3 * o:3 * (o + H * W)].view(3, H, W).cpu().numpy().astype(np.float64)
        d = dep.detach()[o:o + H * W].view(H, W).cpu().numpy().astype(np.float64)
        assert_forward_close(c, d, ref)
    gcs, gds = scenes.linear_loss_weights(310, cams)
    _linear_backward(col, dep, gcs, gds)
    torch.cuda.synchronize()
    grads, g_delta, exclude, g_delta_f = oracle_reference(w.scene, rcams, gcs, gds)
    assert_grads_close(_grads(leaves), grads, exclude, visible=visible_count(w.scene, rcams))
    ref_xi = oracle.pose_tangent_vjp(xi, g_delta)
    assert_pose_close(xt.grad.cpu().numpy(), ref_xi, oracle.pose_tangent_vjp(xi, g_delta_f))
    # away from zero the pull-back is not the identity
    assert np.abs(ref_xi - g_delta).max() > 1e-3 * np.abs(ref_xi).max()


def test_rasterize_directional_finite_difference():
    """(L(theta + h d) - L(theta - h d)) / 2h through the autograd function in
    FP32 against the directional derivative its backward returns, on the
    tiny scene whose oracle gradient is pinned to FP64 central differences.
    The direction moves every parameter and the camera tangent; it is
    checked first, on the oracle, to cross no discrete decision within h (no
    pixel's skip, stop or clamp changes), where a finite difference of this
    piecewise-smooth loss is valid."""
    w = scenes.tiny_scene(16, n=10, degree=3)
    sc = w.scene
    rng = np.random.default_rng(17)
    R, t = scenes.random_pose(rng, 0.05, 0.05)
    cam = scenes.Camera(32, 24, 30.0, 30.0, 16.0, 12.0, R.astype(np.float32), t.astype(np.float32))
    gC, gD = scenes.linear_loss_weights(18, [cam])
    gC, gD = [gC[0] * 100], [gD[0] * 100]
    xi0 = np.array([0.01, -0.02, 0.015, 0.02, -0.01, 0.03])
    drng = np.random.default_rng(0)
    d = {f: drng.standard_normal(getattr(sc, f).shape) for f in FIELDS}
    dxi = drng.standard_normal(6) * 0.5
    h = 1e-4

    # the direction is smooth at h on the oracle (FP64)
    def oracle_loss(sgn):
        s2 = scenes.Scene(*[getattr(sc, f).astype(np.float64) + sgn * h * d[f] for f in FIELDS],
                          sc.sh_degree)
        c = oracle.retract_camera(cam, xi0 + sgn * h * dxi, round32=False)
        return oracle.linear_loss([oracle.render(s2, c)], gC, gD)
    c0 = oracle.retract_camera(cam, xi0, round32=False)
    og, odel = oracle.backward(sc, [c0], gC, gD)
    oan = sum(float((og[f] * d[f].reshape(og[f].shape)).sum()) for f in FIELDS) + \
        float(oracle.pose_tangent_vjp(xi0, odel)[0] @ dxi)
    ofd = (oracle_loss(1) - oracle_loss(-1)) / (2 * h)
    assert abs(ofd - oan) <= 1e-5 * abs(oan), (ofd, oan)

    print("autograd directional finite difference", flush=True)
    ct = gsr.cameras_tensor([cam], DEV)
    wh = [(cam.width, cam.height)]
    gct, gdt = t32(gC[0].reshape(-1)), t32(gD[0].reshape(-1))
    base = gsr.Gaussians.from_scene(sc, DEV)
    dt = {f: t32(d[f].reshape(getattr(base, f).shape)) for f in FIELDS}

    def gpu_loss(sgn, grad=False):
        leaves = [(getattr(base, f).double() + sgn * h * dt[f].double()).float()
                  .requires_grad_(grad) for f in FIELDS]
        xt = t32(xi0 + sgn * h * dxi).reshape(1, 6).requires_grad_(grad)
        col, dep, _ = gsr.rasterize(*leaves, ct, wh, sc.sh_degree, pose_tangent=xt)
        loss = (col.double() * gct.double()).sum() + (dep.double() * gdt.double()).sum()
        if grad:
            loss.backward()
            an = sum(float((x.grad.double() * dt[f].double()).sum()) for f, x in zip(FIELDS, leaves))
            an += float((xt.grad.double().cpu().numpy()[0] * dxi).sum())
            return float(loss), an
        return float(loss)

    with torch.no_grad():
        lp, lm = gpu_loss(1), gpu_loss(-1)
    _, an = gpu_loss(0, grad=True)
    fd = (lp - lm) / (2 * h)
    print(f"directional derivative {an:.6f}, FP32 central difference {fd:.6f}, oracle {oan:.6f}")
    assert abs(fd - an) <= 2e-2 * abs(an), (fd, an)
    assert abs(an - oan) <= 1e-3 * abs(oan), (an, oan)


def test_rasterizer_grows_pair_capacity_and_reuses_workspaces():
    """A Rasterizer planned for 16 pairs re-plans on the overflow of its
    first forward and renders what a plan with the exact capacity renders;
    the next calls take their workspace from the pool."""
    w = workload(1)
    cam = w.cameras[0]
    ct = gsr.cameras_tensor([cam], DEV)
    rz = gsr.Rasterizer([(cam.width, cam.height)], 0, pair_capacity=16)
    leaves = _leaves(w.scene)
    col, dep, T = rz(*leaves, ct)
    assert rz.capacity > 16 and not rz.overflowed()
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    cap = gsr.required_pairs(*g.tensors(), ct, [(cam.width, cam.height)], 0, (16, 16))
    plan = gsr.Plan(w.scene.n, 0, [(cam.width, cam.height)], pair_capacity=cap)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    gsr.preprocess(plan, ws, g, ct)
    gsr.bin_sort(plan, ws)
    gsr.render_fwd(plan, ws, ct, fr)
    torch.cuda.synchronize()
    assert torch.equal(col.detach(), fr.color) and torch.equal(dep.detach(), fr.depth)
    (col.sum() + dep.sum()).backward()
    assert len(rz._free) == 1
    ws_ptr = rz._free[0].data_ptr()
    with torch.no_grad():
        col2, _, _ = rz(*leaves, ct)
    assert len(rz._free) == 1 and rz._free[0].data_ptr() == ws_ptr
    assert torch.equal(col2, fr.color)
