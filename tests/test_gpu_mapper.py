"""The mapping loop with densification (Sec. IV-A): statistics after every
iteration, clone / split / prune every few iterations, then a re-plan and a
re-capture for the new Gaussian count.  The first iteration after each
re-plan (a replay of the new graph) must equal a freshly planned eager
iteration on copies of the new pool and Adam state (parameters, moments,
images, loss bit for bit), and its image the separate calls on the new
pool."""
import numpy as np
import pytest
import torch

import paper_2410_00486_amd as gsr
from paper_2410_00486_amd import _lib as L
from synth import scenes

from gpu_common import DEV, t32

pytestmark = pytest.mark.gpu

LRS = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}


def _copy(g):
    return gsr.Gaussians(*[x.clone() for x in g.tensors()], g.sh_degree)


def test_densify_replan_recapture_equals_fresh_iteration():
    w = scenes.slab_128x96()
    cam = w.cameras[0]
    ct = gsr.cameras_tensor([cam], DEV)
    trgb = t32(w.target_rgb[0].reshape(-1))
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    # every visible Gaussian is densified (tau_p 0) and those under 0.3
    # opacity are pruned, so that the count moves both ways
    mp = gsr.Mapper(g, ct, [(cam.width, cam.height)], trgb, None, LRS, tile=(16, 16),
                    densify_every=2, tau_p=0.0, eps_alpha=0.3, extent=4.0, seed=3)
    counts = [mp.g.n]
    for rnd in range(3):
        while mp.replans == rnd:   # until the next densification and re-plan
            mp.step()
        torch.cuda.synchronize()
        n = mp.g.n
        counts.append(n)
        print(f"round {rnd}: {counts[-2]} -> {n} Gaussians, replans {mp.replans}", flush=True)
        assert mp.replans == rnd + 1
        # the state the next replay starts from, copied
        g0, m0, v0 = _copy(mp.g), _copy(mp.it.m), _copy(mp.it.v)
        step0 = mp.it.step_dev.clone()
        s0 = int(step0.item())
        cap = mp.plan.pair_capacity
        mp.step()
        torch.cuda.synchronize()
        assert mp.plan.flags_of(mp.it.ws)[L.F_OVERFLOW] == 0
        g1 = _copy(g0)  # for the separate calls below
        # a fresh, eagerly enqueued iteration on the copies
        plan = gsr.Plan(n, 0, [(cam.width, cam.height)], tile=(16, 16), lds_batch=64,
                        flags=L.GS_FUSED_L1, pair_capacity=cap)
        ref = gsr.Iteration(plan, g0, ct, target_rgb=trgb, adam_lrs=LRS, adam_state=(m0, v0, step0))
        ref.enqueue()
        torch.cuda.synchronize()
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(mp.g, f), getattr(ref.g, f)), (rnd, f)
            assert torch.equal(getattr(mp.it.m, f), getattr(ref.m, f)), (rnd, f)
            assert torch.equal(getattr(mp.it.v, f), getattr(ref.v, f)), (rnd, f)
        assert torch.equal(mp.it.frame.color, ref.frame.color)
        assert torch.equal(mp.it.frame.loss, ref.frame.loss)
        assert int(mp.it.step_dev.item()) == s0 + 1 == int(ref.step_dev.item())
        # the image of the new pool by the separate calls
        plan1 = gsr.Plan(n, 0, [(cam.width, cam.height)], tile=(16, 16), pair_capacity=cap)
        ws1 = plan1.new_workspace(DEV)
        fr1 = gsr.Frame(plan1, DEV)
        gsr.preprocess(plan1, ws1, g1, ct)
        gsr.bin_sort(plan1, ws1)
        gsr.render_fwd(plan1, ws1, ct, fr1)
        torch.cuda.synchronize()
        assert torch.equal(fr1.color, ref.frame.color)
    assert len(set(counts)) > 2
    mp.close()
