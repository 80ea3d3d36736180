"""Spatial layout of the pool: gs_spatial_order against Morton codes computed
with numpy (same float32 normalisation), a bijection, stable among equal
codes; gs_permute_gaussians against torch indexing; a permuted pool renders
the same image bits; the mapping loop keeps its pool ordered."""
import numpy as np
import pytest
import torch

import paper_2410_00486_amd as gsr
from synth import scenes

from gpu_common import DEV, t32

pytestmark = pytest.mark.gpu


def _morton_np(means):
    m = np.asarray(means, np.float32)
    lo, hi = m.min(0), m.max(0)
    ext = (hi - lo).astype(np.float32)
    t = np.where(ext > 0, (m - lo) / np.where(ext > 0, ext, 1), 0).astype(np.float32)
    t = np.clip(t, 0, 1).astype(np.float32)
    q = (t * np.float32(1023.0)).astype(np.uint64)
    code = np.zeros(len(m), np.uint64)
    for b in range(10):
        for d in range(3):
            code |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return code


@pytest.mark.parametrize("n", [1, 1000, 100_003])
def test_spatial_order_sorts_morton_codes(n):
    rng = np.random.default_rng(n)
    means = rng.normal(0.0, 2.0, (n, 3)).astype(np.float32)
    means[: n // 10] = means[0]            # equal codes: stable order
    perm = gsr.spatial_order(t32(means)).cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(np.sort(perm), np.arange(n))
    code = _morton_np(means)
    np.testing.assert_array_equal(perm, np.argsort(code, kind="stable"))


def test_permute_and_render_invariance():
    w = scenes.slab_128x96()
    cam = w.cameras[0]
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    perm = gsr.spatial_order(g.means)
    gp = gsr.permute(g, perm)
    idx = perm.to(torch.int64)
    for f in gsr.Gaussians.FIELDS:
        assert torch.equal(getattr(gp, f), getattr(g, f).index_select(0, idx)), f
    ct = gsr.cameras_tensor([cam], DEV)
    wh = [(cam.width, cam.height)]
    out = []
    for gg in (g, gp):
        plan = gsr.Plan(g.n, 0, wh, pair_capacity=1 << 16)
        ws = plan.new_workspace(DEV)
        fr = gsr.Frame(plan, DEV)
        gsr.preprocess(plan, ws, gg, ct)
        gsr.bin_sort(plan, ws)
        gsr.render_fwd(plan, ws, ct, fr)
        out.append((fr.color.clone(), fr.depth.clone()))
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


def test_mapper_keeps_the_pool_ordered():
    w = scenes.slab_128x96()
    cam = w.cameras[0]
    ct = gsr.cameras_tensor([cam], DEV)
    trgb = t32(w.target_rgb[0].reshape(-1))
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    lrs = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    mp = gsr.Mapper(g, ct, [(cam.width, cam.height)], trgb, None, lrs, tile=(16, 16),
                    densify_every=2, tau_p=0.0, eps_alpha=0.3, extent=4.0, seed=3,
                    spatial_order=True)
    for _ in range(4):        # re-plans (and re-orders) after steps 2 and 4
        mp.step()
    torch.cuda.synchronize()
    assert mp.replans == 2
    code = _morton_np(mp.g.means.cpu().numpy())
    assert (np.diff(code.astype(np.int64)) >= 0).all()
    mp.close()
