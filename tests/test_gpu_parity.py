"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Forward colour and depth must match within 1e-5 relative (+1e-7 absolute);
gradients within 1e-3 relative (+1e-3 of the tensor's rms) per element and
1e-4 in norm.  Pixels where the oracle sees a discrete decision (alpha clamp,
1/255 skip, 1e-4 stop) within a relative 1e-5 of its threshold are excluded
and counted; Gaussians whose own decision is that close, or whose oracle
gradient moves by more than a quarter of its tolerance when those decisions
take the other branch, are excluded from the gradient check (fewer than 1 %
of the visible ones).  Integer and index work (tile boxes, pair
counts, the sorted pair list, `last`) must be bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_00486_amd as gsr
from paper_2410_00486_amd import _lib as L
from synth import scenes

from gpu_common import (DEV, assert_forward_close, assert_grads_close, assert_pose_close,
                        decided_target, grads_np, oracle_reference, run_gpu, t32, view_images, visible_count,
                        workload)

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ preprocess

@pytest.mark.parametrize("cfg", [1, 3])
def test_preprocess_records_match_oracle(cfg):
    w = workload(cfg)
    cam = w.cameras[0]
    print(f"preprocess parity workload {cfg}", flush=True)
    it = run_gpu(w.scene, [cam])
    plan, ws = it.plan, it.ws
    n = w.scene.n
    ref = oracle.preprocess(w.scene, cam)
    tt = plan.region(ws, L.GS_WS_TILES_TOUCHED, torch.int32, n).cpu().numpy()
    rec = plan.region(ws, L.GS_WS_RECORDS, torch.uint8, n * 64).cpu().numpy().reshape(n, 64)
    rects = plan.region(ws, L.GS_WS_RECTS, torch.int16, 4 * n).cpu().numpy().reshape(n, 4).view(np.uint16)
    vis = ref["status"] == 1
    edge = ref["near_edge"] != 0
    np.testing.assert_array_equal((tt > 0), vis)
    np.testing.assert_array_equal(tt[~edge], ref["tiles_touched"][~edge])
    np.testing.assert_array_equal(rects[vis & ~edge].astype(np.int32), ref["rect"][vis & ~edge])
    d = rec[vis, :16].copy().view(np.float64).reshape(-1, 2)
    f = rec[vis, 16:52].copy().view(np.float32).reshape(-1, 9).astype(np.float64)
    np.testing.assert_allclose(d, ref["mean2d"][vis], rtol=1e-12, atol=1e-9)
    # the exponent's eigen form, in FP32: with the oracle's conic
    # [[a, b], [b, c]], log2(e)/2 d^T Q d = s1 (dx + t dy)^2 + s2 (dy - t dx)^2,
    # |t| <= 1; the conic it stands for is compared (the form is not unique
    # when the footprint's axes lie at 45 degrees), to a few FP32 roundings
    con = ref["conic"][vis]
    t, s1, s2 = f[:, 0], f[:, 1], f[:, 2]
    assert (np.abs(t) <= 1.0).all() and (s1 > 0).all() and (s2 > 0).all()
    got = np.stack([s1 + s2 * t * t, t * (s1 - s2), s1 * t * t + s2], axis=1) / (0.5 * np.log2(np.e))
    err = np.abs(got - con) / np.abs(con).max(axis=1, keepdims=True)
    assert err.max() <= 1e-6, err.max()
    np.testing.assert_allclose(f[:, 3], np.log2(ref["opacity"][vis]), rtol=2e-7, atol=1e-7)
    np.testing.assert_array_equal(f[:, 4], ref["depth32"][vis])
    np.testing.assert_allclose(f[:, 5:8], ref["rgb"][vis], rtol=1.2e-7, atol=1e-12)
    np.testing.assert_allclose(f[:, 8], ref["opacity"][vis], rtol=1.2e-7)
    flags = plan.flags_of(ws)
    assert flags[L.F_VISIBLE] == vis.sum() and flags[L.F_NONFINITE] == 0


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_three_sigma_cutoff_matches_oracle(tile):
    """The comparison-only 3-sigma tile box (GS_CUTOFF_3SIGMA): boxes and
    pair counts bit-exact, the image within the forward tolerance and `last`
    bit-exact against the oracle's 3-sigma branch."""
    w = workload(1)
    cam = w.cameras[0]
    ref = oracle.render(w.scene, cam, tile, cutoff="3sigma")
    pre = ref["pre"]
    print(f"3-sigma cutoff, tile {tile}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile, flags=L.GS_CUTOFF_3SIGMA,
                 capacity=int(pre["tiles_touched"].astype(np.int64).sum()) + 64)
    plan, ws = it.plan, it.ws
    n = w.scene.n
    assert plan.flags_of(ws)[L.F_OVERFLOW] == 0
    rects = plan.region(ws, L.GS_WS_RECTS, torch.int16, 4 * n).cpu().numpy().reshape(n, 4).view(np.uint16)
    tt = plan.region(ws, L.GS_WS_TILES_TOUCHED, torch.int32, n).cpu().numpy()
    vis = pre["status"] == 1
    ok = vis & (pre["near_edge"] == 0)
    np.testing.assert_array_equal(tt > 0, vis)
    np.testing.assert_array_equal(rects[ok].astype(np.int32), pre["rect"][ok])
    np.testing.assert_array_equal(tt[ok], pre["tiles_touched"][ok])
    ex = oracle.preprocess(w.scene, cam, tile)
    assert int(pre["tiles_touched"].sum()) != int(ex["tiles_touched"].sum())
    col, dep, _, last = view_images(it, 0)
    assert_forward_close(col, dep, ref)
    okp = ref["flag"] == 0
    np.testing.assert_array_equal(last[okp], ref["last"][okp])


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("n,bits", [(1, 40), (17, 38), (4096, 44), (4097, 44), (100_003, 48),
                                    (1_000_000, 52), (65_536, 64), (1_500_007, 46)])
def test_sort_pairs_bit_exact(n, bits):
    keys, vals = scenes.random_keys(n, n, max(1, bits - 32))
    if bits == 64:
        keys ^= np.uint64(1) << np.uint64(63)
    kt = torch.from_numpy(keys.view(np.int64).copy()).to(DEV)
    vt = torch.from_numpy(vals.view(np.int32).copy()).to(DEV)
    gsr.sort_pairs(kt, vt, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint64), keys[order])
    np.testing.assert_array_equal(vt.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("cfg,tile", [(1, (16, 16)), (1, (8, 8)), (3, (16, 8)), (2, (16, 16))])
def test_bin_sort_matches_oracle(cfg, tile):
    w = workload(cfg)
    cam = w.cameras[0]
    print(f"bin_sort parity workload {cfg} tile {tile}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile)
    plan, ws = it.plan, it.ws
    pre = oracle.preprocess(w.scene, cam, tile)
    assert not (pre["near_edge"] != 0).any(), "a rect edge is ambiguous; pick another seed"
    keys, vals, ranges = oracle.sort_pairs(pre, cam, tile)
    fl = plan.flags_of(ws)
    P = int(fl[L.F_PAIRS])
    assert fl[L.F_OVERFLOW] == 0 and P == keys.shape[0]
    gk = plan.region(ws, L.GS_WS_SORTED_KEYS, torch.int64, P).cpu().numpy().view(np.uint64)
    gr = plan.region(ws, L.GS_WS_SORTED_RECS, torch.int32, P).cpu().numpy()
    grg = plan.region(ws, L.GS_WS_RANGES, torch.int32, ranges.size).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys)
    np.testing.assert_array_equal(gr, vals.astype(np.int32))
    np.testing.assert_array_equal(grg, ranges)


@pytest.mark.parametrize("tile,n", [((16, 16), 6000), ((8, 8), 3000), ((8, 8), 300),
                                    ((16, 16), 20000)])
def test_bin_sort_long_tile_list(tile, n):
    """n pairs in one tile: each path of the per-tile sort (300: bitonic in
    one wavefront's LDS; 3000 and 6000: bitonic in a block's LDS (up to 8192); 20000:
    bitonic in place in global memory) against the oracle's order."""
    w = scenes.crowded_scene(1, n=n)
    cam = w.cameras[0]
    print(f"bin_sort long list tile {tile} n {n}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile)
    plan, ws = it.plan, it.ws
    pre = oracle.preprocess(w.scene, cam, tile)
    assert not (pre["near_edge"] != 0).any()
    keys, vals, ranges = oracle.sort_pairs(pre, cam, tile)
    r = ranges.reshape(-1, 2).astype(np.int64)
    assert (r[:, 1] - r[:, 0]).max() == n
    fl = plan.flags_of(ws)
    P = int(fl[L.F_PAIRS])
    assert fl[L.F_OVERFLOW] == 0 and P == keys.shape[0]
    gk = plan.region(ws, L.GS_WS_SORTED_KEYS, torch.int64, P).cpu().numpy().view(np.uint64)
    gr = plan.region(ws, L.GS_WS_SORTED_RECS, torch.int32, P).cpu().numpy()
    grg = plan.region(ws, L.GS_WS_RANGES, torch.int32, ranges.size).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys)
    np.testing.assert_array_equal(gr, vals.astype(np.int32))
    np.testing.assert_array_equal(grg, ranges)


@pytest.mark.parametrize("flags", [0, L.GS_SPLAT_BWD])
def test_long_tile_list_forward_backward(flags):
    """Forward and both backward variants on a 6000-splat tile list."""
    w = scenes.crowded_scene(2)
    cam = w.cameras[0]
    gc, gd = scenes.linear_loss_weights(7, [cam])
    print(f"long list forward/backward flags {flags}", flush=True)
    it = run_gpu(w.scene, [cam], lds=64, dL_dcolor=gc, dL_ddepth=gd, flags=flags)
    ref = oracle.render(w.scene, cam)
    col, dep, _, _ = view_images(it, 0)
    assert_forward_close(col, dep, ref)
    grads, _, exclude, _ = oracle_reference(w.scene, [cam], gc, gd)
    assert_grads_close(grads_np(it), grads, exclude, visible=visible_count(w.scene, [cam]))


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("cfg", [1, 3, 2])
def test_forward_matches_oracle(cfg):
    w = workload(cfg)
    cam = w.cameras[0]
    print(f"forward parity workload {cfg}", flush=True)
    it = run_gpu(w.scene, [cam])
    col, dep, T, last = view_images(it, 0)
    ref = oracle.render(w.scene, cam)
    nflag = assert_forward_close(col, dep, ref)
    ok = ref["flag"] == 0
    np.testing.assert_array_equal(last[ok], ref["last"][ok])
    # transmittance: relative error bounded by the conditioning of 1 - alpha
    np.testing.assert_allclose(T[ok], ref["T_final"][ok], rtol=2e-4, atol=1e-7)
    print(f"workload {cfg}: {nflag} flagged pixels of {ok.size}")


def test_forward_tile_shapes_identical():
    w = workload(3)
    cam = w.cameras[0]
    outs = [view_images(run_gpu(w.scene, [cam], tile=t), 0) for t in [(16, 16), (16, 8), (8, 8)]]
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
        np.testing.assert_array_equal(o[2], outs[0][2])


# ------------------------------------------------------------------ backward

def _bwd_case(cfg, tile=(16, 16), lds=256, pose=False, flags=0):
    w = workload(cfg)
    cam = w.cameras[0]
    gc, gd = scenes.linear_loss_weights(100 + cfg, [cam])
    print(f"backward parity workload {cfg} tile {tile} lds {lds} flags {flags}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile, lds=lds, dL_dcolor=gc, dL_ddepth=gd, pose=pose,
                 flags=flags)
    grads, pose_ref, exclude, pose_flip = oracle_reference(w.scene, [cam], gc, gd, tile)
    return it, grads, (pose_ref, pose_flip), exclude


@pytest.mark.parametrize("cfg,tile,lds", [(1, (16, 16), 256), (1, (8, 8), 64), (1, (16, 8), 128),
                                          (3, (16, 16), 256), (2, (16, 16), 128)])
def test_backward_matches_oracle(cfg, tile, lds):
    it, grads, _, exclude = _bwd_case(cfg, tile, lds)
    visible = visible_count(workload(cfg).scene, workload(cfg).cameras[:1], tile)
    rep = assert_grads_close(grads_np(it), grads, exclude, visible=visible)
    print(f"workload {cfg}: excluded {int(exclude.sum())} Gaussians; (max err/tol, rel norm) {rep}")


@pytest.mark.parametrize("cfg,tile,lds", [(1, (16, 16), 256), (1, (8, 8), 32), (1, (16, 8), 96),
                                          (3, (16, 16), 128), (2, (8, 8), 64), (2, (16, 16), 256)])
def test_splat_backward_matches_oracle(cfg, tile, lds):
    """Splat-wise backward (buckets of 64 splats, stored pixel states) against
    the oracle; its forward (which also stores the states) must equal the
    plain forward bit for bit."""
    it, grads, _, exclude = _bwd_case(cfg, tile, lds, flags=L.GS_SPLAT_BWD)
    w = workload(cfg)
    visible = visible_count(w.scene, w.cameras[:1], tile)
    rep = assert_grads_close(grads_np(it), grads, exclude, visible=visible)
    print(f"workload {cfg}: excluded {int(exclude.sum())} Gaussians; (max err/tol, rel norm) {rep}")
    plain = run_gpu(w.scene, [w.cameras[0]], tile=tile, lds=lds)
    for k in range(4):
        np.testing.assert_array_equal(view_images(it, 0)[k], view_images(plain, 0)[k])


def test_splat_backward_multi_view_and_pose():
    scene, cams = _multi_view_workload()
    gcs, gds = scenes.linear_loss_weights(47, cams)
    print("splat-wise backward, 4 views, pose", flush=True)
    it = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds, pose=True,
                 flags=L.GS_SPLAT_BWD | L.GS_PERSISTENT)
    grads, poses, exclude, poses_f = oracle_reference(scene, cams, gcs, gds)
    assert_grads_close(grads_np(it), grads, exclude, visible=visible_count(scene, cams))
    assert_pose_close(it.dL_dpose.cpu().numpy(), poses, poses_f)


def test_pose_gradient_matches_oracle():
    """GPU camera tangent vs the oracle at 640x480 / 150k, and on the small
    scene whose oracle tangent is checked against FP64 central differences
    in the CPU pins (an FP32 finite difference of a 150k-Gaussian image is not
    a valid check: the 1/255 skip and the 1e-4 stop make the loss jump)."""
    it, grads, (pose_ref, pose_flip), exclude = _bwd_case(3, pose=True)
    assert_grads_close(grads_np(it), grads, exclude,
                       visible=visible_count(workload(3).scene, workload(3).cameras))
    assert_pose_close(it.dL_dpose.cpu().numpy(), pose_ref, pose_flip)
    # the FD-pinned small scene (same construction as the CPU pin)
    w = scenes.tiny_scene(16, n=10, degree=3)
    rng = np.random.default_rng(17)
    R, t = scenes.random_pose(rng, 0.05, 0.05)
    cam = scenes.Camera(32, 24, 30.0, 30.0, 16.0, 12.0, R.astype(np.float32), t.astype(np.float32))
    gC, gD = scenes.linear_loss_weights(18, [cam])
    gC, gD = [gC[0] * 100], [gD[0] * 100]
    it2 = run_gpu(w.scene, [cam], dL_dcolor=gC, dL_ddepth=gD, pose=True)
    grads2, pose2 = oracle.backward(w.scene, [cam], gC, gD)
    got2 = it2.dL_dpose.cpu().numpy().astype(np.float64)[0]
    assert np.linalg.norm(got2 - pose2[0]) <= 1e-3 * np.linalg.norm(pose2[0]), (got2, pose2[0])
    assert_grads_close(grads_np(it2), grads2)


def test_fused_l1_matches_oracle():
    """The fused L1 RGB + 0.1 L1 depth loss and its gradients against the
    oracle, with a target whose every residual is decided at FP32 accuracy
    (the render of the perturbed scene, residuals under 1e-4 pushed out to
    1e-4), so that no L1 sign is ambiguous."""
    w = workload(2)
    cam = w.cameras[0]
    tgt = oracle.render(w.target_scene, cam)
    ref = oracle.render(w.scene, cam)
    trgb = decided_target(ref["color"], tgt["color"])
    tdep = decided_target(ref["depth"], tgt["depth"])
    it = run_gpu(w.scene, [cam], flags=L.GS_FUSED_L1, target_rgb=[trgb], target_depth=[tdep],
                 lambda_depth=0.1)
    loss, gC, gD = oracle.l1_loss_and_grads(ref["color"], ref["depth"], trgb, tdep, 0.1)
    got_loss = float(it.frame.loss.cpu()[0])
    assert abs(got_loss - loss) <= 1e-5 * abs(loss)
    grads, _, exclude, _ = oracle_reference(w.scene, [cam], [gC], [gD])
    rep = assert_grads_close(grads_np(it), grads, exclude, visible=visible_count(w.scene, [cam]))
    print(f"excluded {int(exclude.sum())}; (max err/tol, rel norm) {rep}")


# ------------------------------------------------------------------ Adam

def test_adam_matches_oracle():
    rng = np.random.default_rng(3)
    n = 100_003
    shapes = {"means": (n, 3), "log_scales": (n, 3), "quats": (n, 4), "opacity_logits": (n,),
              "sh": (n, 16, 3)}
    lrs = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    P = {k: rng.standard_normal(s) for k, s in shapes.items()}
    mk = lambda d: gsr.Gaussians(*[t32(d[k]) for k in gsr.Gaussians.FIELDS], 3)
    params, m, v = mk(P), mk({k: np.zeros(s) for k, s in shapes.items()}), mk({k: np.zeros(s) for k, s in shapes.items()})
    grads = mk({k: rng.standard_normal(s) for k, s in shapes.items()})
    groups = gsr.adam_groups(params, grads, m, v, lrs, opacity_reg=True)
    ref = {k: (P[k].astype(np.float32).astype(np.float64), np.zeros(shapes[k]), np.zeros(shapes[k])) for k in shapes}
    for step in (1, 2, 3):
        gnp = {k: rng.standard_normal(shapes[k]).astype(np.float32) for k in shapes}
        for k in shapes:
            getattr(grads, k).copy_(t32(gnp[k]))
        gsr.adam_step(groups, step, lambda_o=0.001, reg_count=n)
        for k in shapes:
            p0, m0, v0 = ref[k]
            g = gnp[k].astype(np.float64)
            if k == "opacity_logits":
                g = g + oracle.opacity_reg_grad(p0, 0.001, n)
            ref[k] = oracle.adam_step(p0, g, m0, v0, step, lrs[k])
    torch.cuda.synchronize()
    for k in shapes:
        p, mm, vv = ref[k]
        np.testing.assert_allclose(getattr(params, k).cpu().numpy(), p, rtol=2e-6, atol=1e-7)
        np.testing.assert_allclose(getattr(m, k).cpu().numpy(), mm, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(getattr(v, k).cpu().numpy(), vv, rtol=1e-5, atol=1e-8)


# ------------------------------------------------------------------ batching, graphs, modes

def _multi_view_workload():
    w = workload(4, n=120_000, n_views=4)
    return w.scene, w.cameras


def test_batched_equals_per_view():
    scene, cams = _multi_view_workload()
    gcs, gds = scenes.linear_loss_weights(44, cams)
    batched = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds, pose=True)
    gb = grads_np(batched)
    acc = None
    for v, cam in enumerate(cams):
        single = run_gpu(scene, [cam], dL_dcolor=[gcs[v]], dL_ddepth=[gds[v]], pose=True)
        for k in range(4):
            np.testing.assert_array_equal(view_images(single, 0)[k], view_images(batched, v)[k])
        np.testing.assert_allclose(single.dL_dpose.cpu().numpy()[0], batched.dL_dpose.cpu().numpy()[v],
                                   rtol=1e-4, atol=1e-6 * np.abs(batched.dL_dpose.cpu().numpy()).max())
        gv = grads_np(single)
        acc = gv if acc is None else {k: acc[k] + gv[k] for k in acc}
    for k in gb:
        scale = np.abs(gb[k]).max()
        np.testing.assert_allclose(gb[k], acc[k], rtol=1e-4, atol=1e-6 * scale)


def test_batched_matches_oracle_multi_view():
    scene, cams = _multi_view_workload()
    gcs, gds = scenes.linear_loss_weights(45, cams)
    it = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds, pose=True, flags=L.GS_PERSISTENT)
    for v, cam in enumerate(cams):
        ref = oracle.render(scene, cam)
        col, dep, _, _ = view_images(it, v)
        assert_forward_close(col, dep, ref)
    grads, poses, exclude, poses_f = oracle_reference(scene, cams, gcs, gds)
    assert_grads_close(grads_np(it), grads, exclude, visible=visible_count(scene, cams))
    assert_pose_close(it.dL_dpose.cpu().numpy(), poses, poses_f)


def test_multi_view_without_pose_matches_pose_path_and_oracle():
    """Several views without the camera tangent take the projection
    backward in three launches (a thread per visible record, then the
    projection and colour halves per Gaussian).  Against the one-thread-per-
    Gaussian form that also computes the tangent: the same sums in the same
    view order, only the mean gradient adds its two halves in another order
    (within a few ulp); and against the oracle."""
    scene, cams = _multi_view_workload()
    gcs, gds = scenes.linear_loss_weights(48, cams)
    print("4 views 120k without camera tangent: against the tangent form and the oracle", flush=True)
    a = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds)
    b = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds, pose=True)
    ga, gb = grads_np(a), grads_np(b)
    for f in ga:
        scale = float(np.abs(gb[f]).max())
        np.testing.assert_allclose(ga[f], gb[f], rtol=1e-6, atol=1e-9 * scale, err_msg=f)
    grads, _, exclude, _ = oracle_reference(scene, cams, gcs, gds)
    assert_grads_close(ga, grads, exclude, visible=visible_count(scene, cams))


def test_persistent_equals_plain():
    scene, cams = _multi_view_workload()
    gcs, gds = scenes.linear_loss_weights(46, cams)
    a = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds)
    b = run_gpu(scene, cams, dL_dcolor=gcs, dL_ddepth=gds, flags=L.GS_PERSISTENT, chunk=4)
    for v in range(len(cams)):
        for k in range(4):
            np.testing.assert_array_equal(view_images(a, v)[k], view_images(b, v)[k])
    ga, gb = grads_np(a), grads_np(b)
    for k in ga:
        np.testing.assert_array_equal(ga[k], gb[k])


@pytest.mark.parametrize("flags", [L.GS_FUSED_L1, L.GS_FUSED_L1 | L.GS_SPLAT_BWD])
def test_graph_replay_equals_eager(flags):
    w = workload(1)
    cam = w.cameras[0]
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    tgt = t32(w.target_rgb[0].reshape(-1))

    def make():
        g = gsr.Gaussians.from_scene(w.scene, DEV)
        plan = gsr.Plan(w.scene.n, 0, [(cam.width, cam.height)], flags=flags,
                        pair_capacity=1 << 16)
        return gsr.Iteration(plan, g, gsr.cameras_tensor([cam], DEV), target_rgb=tgt,
                             adam_lrs=lrs, lambda_o=0.001)

    eager, graphed = make(), make()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graphed.capture(s)
    for step in range(3):
        eager.enqueue()
        torch.cuda.synchronize()
        _ = (eager.frame.color * 2).sum().item()      # unrelated eager work in between
        with torch.cuda.stream(s):
            graphed.replay(s)
        s.synchronize()
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(eager.g, f), getattr(graphed.g, f)), (step, f)
        assert torch.equal(eager.frame.color, graphed.frame.color)
        assert torch.equal(eager.frame.loss, graphed.frame.loss)
    assert int(graphed.step_dev.item()) == 3
    graphed.close()


@pytest.mark.parametrize("lambda_o,degree", [(0.0, 3), (0.001, 3), (0.0, 2), (0.0, 0)])
def test_iteration_sparse_adam_equals_separate_calls(lambda_o, degree):
    """One-view iteration with Adam (gradients of Gaussians without pairs are
    not written; Adam takes them as zero) against the separate calls with
    fully written gradients: parameters and moments bit for bit."""
    w = workload(3)  # 640x480 view of a 150k room: most Gaussians have no pairs
    cam = w.cameras[0]
    K = (degree + 1) ** 2
    sc = w.scene
    scene = scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits,
                         np.ascontiguousarray(sc.sh[:, :K]), degree)
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    rng = np.random.default_rng(9)
    tgt = t32(rng.uniform(0.0, 1.0, (3, cam.height, cam.width)).reshape(-1))
    cams = gsr.cameras_tensor([cam], DEV)
    g1 = gsr.Gaussians.from_scene(scene, DEV)
    # headroom for the second iteration, whose parameters Adam has moved
    cap = int(gsr.required_pairs(*g1.tensors(), cams, [(cam.width, cam.height)], degree,
                                 (16, 16)) * 1.2) + 64
    plan = gsr.Plan(scene.n, degree, [(cam.width, cam.height)], flags=L.GS_FUSED_L1,
                    pair_capacity=cap)
    it = gsr.Iteration(plan, g1, cams, target_rgb=tgt, adam_lrs=lrs, lambda_o=lambda_o)
    # stale, non-zero gradient buffers must not leak into the step
    for x in it.grads.tensors():
        x.fill_(7.0)
    it.enqueue()
    g2 = gsr.Gaussians.from_scene(scene, DEV)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    grads, m, v = g2.zeros_like(), g2.zeros_like(), g2.zeros_like()
    gsr.preprocess(plan, ws, g2, cams)
    gsr.bin_sort(plan, ws)
    gsr.render_fwd(plan, ws, cams, fr, tgt)
    gsr.render_bwd(plan, ws, g2, cams, fr, grads, target_rgb=tgt)
    groups = gsr.adam_groups(g2, grads, m, v, lrs, lambda_o != 0.0)
    gsr.adam_step(groups, 1, lambda_o=lambda_o, reg_count=g2.n)
    torch.cuda.synchronize()
    assert int(plan.flags_of(it.ws)[L.F_VISIBLE]) < g1.n  # some Gaussians have no pairs
    for f in gsr.Gaussians.FIELDS:
        assert torch.equal(getattr(g1, f), getattr(g2, f)), f
        assert torch.equal(getattr(it.m, f), getattr(m, f)), f
        assert torch.equal(getattr(it.v, f), getattr(v, f)), f
    # the iteration reduces the loss inside its Adam launch and advances the
    # step counter in its first launch: same loss bits, one step per call
    assert torch.equal(it.frame.loss, fr.loss)
    assert int(it.step_dev.item()) == 1
    it.enqueue()
    torch.cuda.synchronize()
    assert int(plan.flags_of(it.ws)[L.F_OVERFLOW]) == 0
    assert int(it.step_dev.item()) == 2


@pytest.mark.parametrize("lambda_o,degree,extra", [
    (0.0, 3, 0), (0.001, 3, L.GS_RADIX_BIN | L.GS_SPLAT_BWD | L.GS_PERSISTENT),
    (0.001, 1, L.GS_SPLAT_BWD), (0.0, 0, L.GS_RADIX_BIN)])
def test_iteration_several_view_adam_equals_separate_calls(lambda_o, degree, extra):
    """Several views with Adam (the per-record and per-Gaussian projection
    backward, then one Adam launch over every Gaussian) against the separate
    calls, two steps: parameters and moments bit for bit, the loss, the
    step counter once per iteration."""
    scene0, cams_l = _multi_view_workload()
    K = (degree + 1) ** 2
    scene = scenes.Scene(scene0.means, scene0.log_scales, scene0.quats, scene0.opacity_logits,
                         np.ascontiguousarray(scene0.sh[:, :K]), degree)
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    wh = [(c.width, c.height) for c in cams_l]
    cams = gsr.cameras_tensor(cams_l, DEV)
    rng = np.random.default_rng(31)
    npx = sum(w * h for w, h in wh)
    tgt = t32(rng.uniform(0.0, 1.0, 3 * npx))
    tdep = t32(rng.uniform(0.5, 4.0, npx))
    g1 = gsr.Gaussians.from_scene(scene, DEV)
    cap = int(gsr.required_pairs(*g1.tensors(), cams, wh, degree, (16, 16)) * 1.3) + 4096
    flags = L.GS_FUSED_L1 | extra
    plan = gsr.Plan(scene.n, degree, wh, flags=flags, pair_capacity=cap)
    print(f"several-view iteration with Adam: lambda_o {lambda_o} degree {degree} flags {flags}",
          flush=True)
    it = gsr.Iteration(plan, g1, cams, target_rgb=tgt, target_depth=tdep, adam_lrs=lrs,
                       lambda_o=lambda_o)
    g2 = gsr.Gaussians.from_scene(scene, DEV)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    grads, m, v = g2.zeros_like(), g2.zeros_like(), g2.zeros_like()
    groups = gsr.adam_groups(g2, grads, m, v, lrs, lambda_o != 0.0)
    for step in (1, 2):
        it.enqueue()
        gsr.preprocess(plan, ws, g2, cams)
        gsr.bin_sort(plan, ws)
        gsr.render_fwd(plan, ws, cams, fr, tgt, tdep)
        gsr.render_bwd(plan, ws, g2, cams, fr, grads, target_rgb=tgt, target_depth=tdep)
        gsr.adam_step(groups, step, lambda_o=lambda_o, reg_count=g2.n)
        torch.cuda.synchronize()
        assert int(plan.flags_of(it.ws)[L.F_OVERFLOW]) == 0
        assert int(it.step_dev.item()) == step
        assert torch.equal(it.frame.loss, fr.loss), step
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(g1, f), getattr(g2, f)), (step, f)
            assert torch.equal(getattr(it.m, f), getattr(m, f)), (step, f)
            assert torch.equal(getattr(it.v, f), getattr(v, f)), (step, f)
        assert all(bool((x != 0).any()) for x in m.tensors())  # every group stepped


@pytest.mark.parametrize("n,extra", [(300, 0), (3000, 0), (300, L.GS_SPLAT_BWD), (3000, L.GS_SPLAT_BWD)])
def test_iteration_sorting_in_forward_equals_separate_calls(n, extra):
    """A whole iteration lets the forward sort each tile's list (up to 128
    pairs; longer lists by the long-list kernel before it).  Against the
    separate calls, whose binning sorts every list itself: the sorted lists,
    the images, the loss and the Adam step bit for bit, on a view with lists
    of n pairs over a few tiles and short lists elsewhere."""
    w = scenes.crowded_scene(3, n=n)
    cam = w.cameras[0]
    sc = w.scene
    print(f"iteration sorting in forward n {n} flags {extra}", flush=True)
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    rng = np.random.default_rng(11)
    tgt = t32(rng.uniform(0.0, 1.0, (3, cam.height, cam.width)).reshape(-1))
    cams = gsr.cameras_tensor([cam], DEV)
    g1 = gsr.Gaussians.from_scene(sc, DEV)
    cap = gsr.required_pairs(*g1.tensors(), cams, [(cam.width, cam.height)], sc.sh_degree, (16, 16)) + 7
    plan = gsr.Plan(sc.n, sc.sh_degree, [(cam.width, cam.height)], flags=L.GS_FUSED_L1 | extra,
                    pair_capacity=cap)
    it = gsr.Iteration(plan, g1, cams, target_rgb=tgt, adam_lrs=lrs)
    it.enqueue()
    g2 = gsr.Gaussians.from_scene(sc, DEV)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    grads, m, v = g2.zeros_like(), g2.zeros_like(), g2.zeros_like()
    gsr.preprocess(plan, ws, g2, cams)
    gsr.bin_sort(plan, ws)
    gsr.render_fwd(plan, ws, cams, fr, tgt)
    gsr.render_bwd(plan, ws, g2, cams, fr, grads, target_rgb=tgt)
    gsr.adam_step(gsr.adam_groups(g2, grads, m, v, lrs, False), 1)
    torch.cuda.synchronize()
    fl = plan.flags_of(ws)
    P = int(fl[L.F_PAIRS])
    assert fl[L.F_OVERFLOW] == 0 and int(plan.flags_of(it.ws)[L.F_PAIRS]) == P
    T = plan.total_tiles
    rg = plan.region(ws, L.GS_WS_RANGES, torch.int32, 2 * T).cpu().numpy().reshape(T, 2)
    assert (rg[:, 1] - rg[:, 0]).max() == n  # the crowded tiles hold n pairs
    for region, dt, cnt in ((L.GS_WS_SORTED_KEYS, torch.int64, P), (L.GS_WS_SORTED_VALS, torch.int32, P),
                            (L.GS_WS_SORTED_RECS, torch.int32, P), (L.GS_WS_RANGES, torch.int32, 2 * T)):
        assert torch.equal(plan.region(it.ws, region, dt, cnt), plan.region(ws, region, dt, cnt)), region
    for a, b in ((it.frame.color, fr.color), (it.frame.depth, fr.depth), (it.frame.T_final, fr.T_final),
                 (it.frame.last, fr.last), (it.frame.loss, fr.loss)):
        assert torch.equal(a, b)
    for f in gsr.Gaussians.FIELDS:
        assert torch.equal(getattr(g1, f), getattr(g2, f)), f
        assert torch.equal(getattr(it.m, f), getattr(m, f)), f
        assert torch.equal(getattr(it.v, f), getattr(v, f)), f


@pytest.mark.parametrize("extra", [L.GS_SPLAT_BWD, 0])
def test_iteration_equals_separate_calls_full_view(extra):
    """The 1200x680 / 300k view (12,750 tiles): one whole iteration, whose
    forward sorts each tile and composites it from what that wavefront just
    wrote, against the separate calls: sorted lists and every image bit for
    bit.  (Many neighbouring tiles per CU: a read of the fresh records through
    a stale cached line would show here.)"""
    w = scenes.room_1200x680()
    cam = w.cameras[0]
    view_wh = [(cam.width, cam.height)]
    cams = gsr.cameras_tensor([cam], DEV)
    g1 = gsr.Gaussians.from_scene(w.scene, DEV)
    rng = np.random.default_rng(5)
    tgt = t32(rng.uniform(0.0, 1.0, (3, cam.height, cam.width)).reshape(-1))
    print(f"full-view iteration against separate calls, flags {extra}", flush=True)
    cap = int(gsr.required_pairs(*g1.tensors(), cams, view_wh, 3, (8, 8)) * 1.2) + 4096
    plan = gsr.Plan(w.scene.n, 3, view_wh, tile=(8, 8), lds_batch=64, flags=L.GS_FUSED_L1 | extra,
                    pair_capacity=cap)
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    it = gsr.Iteration(plan, g1, cams, target_rgb=tgt, adam_lrs=lrs)
    it.enqueue()
    g2 = gsr.Gaussians.from_scene(w.scene, DEV)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    gsr.preprocess(plan, ws, g2, cams)
    gsr.bin_sort(plan, ws)
    gsr.render_fwd(plan, ws, cams, fr, tgt)
    torch.cuda.synchronize()
    P = int(plan.flags_of(ws)[L.F_PAIRS])
    T = plan.total_tiles
    for region, dt, cnt in ((L.GS_WS_SORTED_KEYS, torch.int64, P), (L.GS_WS_SORTED_VALS, torch.int32, P),
                            (L.GS_WS_SORTED_RECS, torch.int32, P), (L.GS_WS_RANGES, torch.int32, 2 * T)):
        assert torch.equal(plan.region(it.ws, region, dt, cnt), plan.region(ws, region, dt, cnt)), region
    for a, b in ((it.frame.color, fr.color), (it.frame.depth, fr.depth), (it.frame.T_final, fr.T_final),
                 (it.frame.last, fr.last), (it.frame.loss, fr.loss)):
        assert int((a != b).sum().item()) == 0


# ------------------------------------------------------------------ edge cases

def test_empty_scene_and_empty_view():
    w = workload(1)
    cam = w.cameras[0]
    empty = w.scene.subset(np.arange(0))
    it = run_gpu(empty, [cam], capacity=1)
    col, dep, T, last = view_images(it, 0)
    assert (col == 0).all() and (dep == 0).all() and (T == 1).all() and (last == 0).all()
    # camera looking away from every Gaussian
    back = scenes.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                         np.diag([1.0, -1.0, -1.0]).astype(np.float32), np.zeros(3, np.float32),
                         bg=(0.1, 0.2, 0.3))
    gc, gd = scenes.linear_loss_weights(1, [back])
    it = run_gpu(w.scene, [back], capacity=1, dL_dcolor=gc, dL_ddepth=gd)
    col, _, _, _ = view_images(it, 0)
    np.testing.assert_allclose(col[0], 0.1, rtol=0, atol=1e-7)
    g = grads_np(it)
    assert all((g[f] == 0).all() for f in g)


@pytest.mark.parametrize("views,tile", [(1, (16, 16)), (1, (16, 8)), (2, (8, 8))])
def test_zero_upstream_gradient_gives_zero_gradients(views, tile):
    """With dL/dC = dL/dD = 0 every parameter gradient is exactly zero (one
    view: the compact projection backward alone; two views: the per-record
    and per-Gaussian launches).  A launch of the several-view form on a
    one-view plan would write its per-Gaussian sums far outside that plan's
    workspace and leave non-zero values here."""
    w = workload(3)
    cams = [w.cameras[0]] if views == 1 else [w.cameras[0], w.gt_cameras[0]]
    print(f"zero upstream gradient: {views} view(s), tile {tile}", flush=True)
    it = run_gpu(w.scene, cams, tile=tile)
    g = grads_np(it)
    for f in g:
        assert int(np.count_nonzero(g[f])) == 0, f


def test_nonfinite_gaussians_are_culled_and_counted():
    w = workload(1)
    cam = w.cameras[0]
    sc = w.scene.copy()
    sc.means[5, 0] = np.nan
    sc.quats[6] = 0.0
    sc.sh[7, 0, 1] = np.inf
    sc.opacity_logits[8] = -np.inf
    it = run_gpu(sc, [cam])
    assert it.plan.flags_of(it.ws)[L.F_NONFINITE] >= 2
    keep = np.setdiff1d(np.arange(sc.n), [5, 6, 7, 8])
    ref = run_gpu(w.scene.subset(keep), [cam])
    np.testing.assert_array_equal(view_images(it, 0)[0], view_images(ref, 0)[0])


def test_pair_capacity_overflow_is_flagged():
    w = workload(1)
    cam = w.cameras[0]
    it = run_gpu(w.scene, [cam], capacity=100)
    fl = it.plan.flags_of(it.ws)
    assert fl[L.F_OVERFLOW] == 1 and fl[L.F_PAIRS_WANTED] > 100 and fl[L.F_PAIRS] == 0


@pytest.mark.parametrize("views,graph", [(1, False), (1, True), (2, False), (2, True)])
def test_overflow_iteration_leaves_optimizer_state_unchanged(views, graph):
    """A whole iteration whose pairs overflow the plan's capacity: its Adam
    step changes no parameter, moment or step counter (one view: the sparse
    in-iteration Adam; two views: the plain one), eagerly and as graph
    replays."""
    w = workload(1)
    cams = [w.cameras[0]] * views
    wh = [(c.width, c.height) for c in cams]
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    tgt = t32(np.concatenate([w.target_rgb[0].reshape(-1)] * views))
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    plan = gsr.Plan(w.scene.n, 0, wh, flags=L.GS_FUSED_L1, pair_capacity=100)
    it = gsr.Iteration(plan, g, gsr.cameras_tensor(cams, DEV), target_rgb=tgt, adam_lrs=lrs,
                       lambda_o=0.001)
    for k, x in enumerate(it.m.tensors()):
        x.fill_(0.25 * (k + 1))
    for k, x in enumerate(it.v.tensors()):
        x.fill_(0.01 * (k + 1))
    it.step_dev.fill_(5)
    before = [x.clone() for x in g.tensors() + it.m.tensors() + it.v.tensors()]
    s = torch.cuda.Stream()
    if graph:
        with torch.cuda.stream(s):
            it.capture(s)
    for rep in range(2):
        if graph:
            with torch.cuda.stream(s):
                it.replay(s)
            s.synchronize()
        else:
            it.enqueue()
        torch.cuda.synchronize()
        fl = plan.flags_of(it.ws)
        assert fl[L.F_OVERFLOW] == 1 and fl[L.F_PAIRS_WANTED] > 100
        after = g.tensors() + it.m.tensors() + it.v.tensors()
        for a, b in zip(before, after):
            assert torch.equal(a, b), rep
        assert int(it.step_dev.item()) == 5
    it.close()


@pytest.mark.parametrize("flags", [0, L.GS_SPLAT_BWD])
def test_elongated_footprints_match_oracle(flags):
    """Needle-like Gaussians (axis ratios near 100, so 2D conics with
    eigenvalue ratios in the thousands, long axes tens of pixels, every
    orientation): forward and gradients within the same tolerances.  The
    exponent is a sum of squares along the footprint's axes, so its error
    does not grow with the elongation."""
    w = scenes.tiny_scene(41, n=40, width=128, height=96, degree=1, f=120.0)
    sc = w.scene.copy()
    sc.log_scales[:, 0] += np.float32(2.5)
    sc.log_scales[:, 1] -= np.float32(2.0)
    sc.log_scales[:, 2] -= np.float32(2.0)
    cam = w.cameras[0]
    gc, gd = scenes.linear_loss_weights(42, [cam])
    print(f"elongated footprints, flags {flags}", flush=True)
    it = run_gpu(sc, [cam], tile=(8, 8), dL_dcolor=gc, dL_ddepth=gd, flags=flags)
    ref = oracle.render(sc, cam, (8, 8))
    col, dep, _, _ = view_images(it, 0)
    assert_forward_close(col, dep, ref)
    grads, _, exclude, _ = oracle_reference(sc, [cam], gc, gd, (8, 8))
    assert_grads_close(grads_np(it), grads, exclude)


def test_ragged_view_and_large_gaussian_and_sh_degrees():
    for deg in (1, 2):
        w = scenes.tiny_scene(31 + deg, n=40, width=33, height=17, degree=deg, f=25.0)
        sc = w.scene.copy()
        sc.log_scales[0] = np.log(0.6)      # one Gaussian larger than the image
        gc, gd = scenes.linear_loss_weights(9, w.cameras)
        cam = w.cameras[0]
        for tile in [(16, 16), (8, 8)]:
            it = run_gpu(sc, [cam], tile=tile, dL_dcolor=gc, dL_ddepth=gd)
            ref = oracle.render(sc, cam, tile)
            col, dep, _, _ = view_images(it, 0)
            assert_forward_close(col, dep, ref)
            grads, _, exclude, _ = oracle_reference(sc, [cam], gc, gd, tile)
            assert_grads_close(grads_np(it), grads, exclude)
