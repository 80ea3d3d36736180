"""Scheduled batches (Sec. III-C-2, Eqs. (5)-(8)): the keyframe scheduler
picks the views of every iteration, the ids go to a device buffer, and one
captured whole-iteration graph gathers those keyframes' cameras and targets
itself.  Against the same iterations enqueued eagerly with the selected
keyframes copied in by the host: images, losses, parameters and Adam moments
bit for bit at every step, through a refill of the counts (Eq. (8))."""
import numpy as np
import pytest
import torch

import paper_2410_00486_amd as gsr
from paper_2410_00486_amd import _lib as L
from synth import scenes

from gpu_common import DEV

pytestmark = pytest.mark.gpu

LRS = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
TILE = (8, 8)
B = 3


def _pool_targets(w, cams):
    wh = [(c.width, c.height) for c in w.cameras]
    tg = gsr.Gaussians.from_scene(w.target_scene, DEV)
    cap = gsr.required_pairs(*tg.tensors(), cams, wh, 3, TILE) + 4096
    plan = gsr.Plan(w.scene.n, 3, wh, tile=TILE, pair_capacity=cap)
    ws = plan.new_workspace(DEV)
    fr = gsr.Frame(plan, DEV)
    gsr.preprocess(plan, ws, tg, cams)
    gsr.bin_sort(plan, ws)
    gsr.render_fwd(plan, ws, cams, fr)
    torch.cuda.synchronize()
    K = len(w.cameras)
    return fr.color.view(K, -1).clone(), fr.depth.view(K, -1).clone()


def test_scheduled_graph_equals_eager_selection():
    w = scenes.keyframe_pool_640x480()
    K = len(w.cameras)
    pool_cams = gsr.cameras_tensor(w.cameras, DEV).view(K, -1).contiguous()
    pool_rgb, pool_dep = _pool_targets(w, pool_cams)
    wh = [(640, 480)] * B
    g0 = gsr.Gaussians.from_scene(w.scene, DEV)
    cap = int(gsr.required_pairs(*g0.tensors(), pool_cams, [(640, 480)] * K, 3, TILE) * 1.3) + 4096
    flags = L.GS_FUSED_L1 | L.GS_PERSISTENT | L.GS_SPLAT_BWD

    def make(gather):
        g = gsr.Gaussians.from_scene(w.scene, DEV)
        plan = gsr.Plan(w.scene.n, 3, wh, tile=TILE, lds_batch=64, chunk=1, flags=flags,
                        pair_capacity=cap)
        cams = torch.zeros(B * L.GS_CAMERA_FLOATS, dtype=torch.float32, device=DEV)
        trgb = torch.zeros(3 * plan.total_pixels, dtype=torch.float32, device=DEV)
        tdep = torch.zeros(plan.total_pixels, dtype=torch.float32, device=DEV)
        return gsr.Iteration(plan, g, cams, target_rgb=trgb, target_depth=tdep, adam_lrs=LRS,
                             gather=gather)

    pool = gsr.KeyframePool(pool_cams, pool_rgb, pool_dep, B)
    graphed, eager = make(pool), make(None)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graphed.capture(s)
    ks = gsr.KeyframeScheduler(capacity=16, r0=2, d=4)
    for _ in range(K):
        ks.add_keyframe()
    rng = np.random.default_rng(7)
    seen, refills = set(), []
    for step in range(6):
        ids = ks.select_batch(rng.uniform(size=B).tolist())
        assert len(ids) == B
        seen.update(ids)
        print(f"step {step}: keyframes {ids}", flush=True)
        pool.select(ids, s)
        with torch.cuda.stream(s):
            graphed.replay(s)
        s.synchronize()
        idx = torch.tensor(ids, device=DEV, dtype=torch.int64)
        eager.cams.copy_(pool_cams.index_select(0, idx).reshape(-1))
        eager.target_rgb.copy_(pool_rgb.index_select(0, idx).reshape(-1))
        eager.target_depth.copy_(pool_dep.index_select(0, idx).reshape(-1))
        eager.enqueue()
        torch.cuda.synchronize()
        assert graphed.plan.flags_of(graphed.ws)[L.F_OVERFLOW] == 0
        assert torch.equal(graphed.cams, eager.cams)
        assert torch.equal(graphed.target_rgb, eager.target_rgb)
        assert torch.equal(graphed.frame.color, eager.frame.color)
        assert torch.equal(graphed.frame.loss, eager.frame.loss)
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(graphed.g, f), getattr(eager.g, f)), (step, f)
            assert torch.equal(getattr(graphed.m, f), getattr(eager.m, f)), (step, f)
        losses = graphed.frame.loss.cpu().tolist()
        for i, l in zip(ids, losses):
            ks.report(i, l)
        refills.append(ks.refills)
    assert refills[-1] >= 1 and len(seen) == K
    graphed.close()


def test_gather_rejects_mixed_view_sizes():
    plan = gsr.Plan(10, 0, [(64, 48), (32, 24)], pair_capacity=64)
    cams = torch.zeros(2, L.GS_CAMERA_FLOATS, dtype=torch.float32, device=DEV)
    rgb = torch.zeros(2, 3 * 64 * 48, dtype=torch.float32, device=DEV)
    pool = gsr.KeyframePool(cams, rgb, None, 2)
    g = pool.c()
    out = torch.zeros(2 * L.GS_CAMERA_FLOATS, dtype=torch.float32, device=DEV)
    import ctypes
    st = L.lib().gs_gather_views(ctypes.byref(plan.c), ctypes.byref(g), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(rgb.data_ptr()), None, None)
    assert st == L.GS_ERR_INVALID_ARG
