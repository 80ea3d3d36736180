"""GPU parity of the radix binning (GS_RADIX_BIN): the visible records
sorted by depth, their pairs generated in that order, then sorted by tile id.
The lists must equal the oracle's stable (tile, depth, generation) order bit
for bit, and everything downstream must then equal the per-tile binning's
results bit for bit: images, gradients, camera tangents, Adam state.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2410_00486_amd as gsr
from paper_2410_00486_amd import _lib as L
from synth import scenes

from gpu_common import DEV, grads_np, run_gpu, t32, view_images, workload

pytestmark = pytest.mark.gpu

RADIX = L.GS_RADIX_BIN
LRS = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}


def _lists(it):
    plan, ws = it.plan, it.ws
    fl = plan.flags_of(ws)
    P, T = int(fl[L.F_PAIRS]), plan.total_tiles
    out = {}
    for name, reg, dt, n in (("keys", L.GS_WS_SORTED_KEYS, torch.int64, P),
                             ("vals", L.GS_WS_SORTED_VALS, torch.int32, P),
                             ("recs", L.GS_WS_SORTED_RECS, torch.int32, P),
                             ("ranges", L.GS_WS_RANGES, torch.int32, 2 * T)):
        out[name] = plan.region(ws, reg, dt, n).cpu().numpy()
    return fl, out


def _same_iteration(a, b, n_views):
    for v in range(n_views):
        for k in range(4):
            np.testing.assert_array_equal(view_images(a, v)[k], view_images(b, v)[k])
    ga, gb = grads_np(a), grads_np(b)
    for f in ga:
        np.testing.assert_array_equal(ga[f], gb[f])


@pytest.mark.parametrize("cfg,tile", [(1, (16, 16)), (1, (8, 8)), (3, (16, 8)), (2, (8, 8))])
def test_radix_bin_matches_oracle(cfg, tile):
    w = workload(cfg)
    cam = w.cameras[0]
    print(f"radix binning workload {cfg} tile {tile}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile, flags=RADIX)
    pre = oracle.preprocess(w.scene, cam, tile)
    assert not (pre["near_edge"] != 0).any(), "a rect edge is ambiguous; pick another seed"
    keys, vals, ranges = oracle.sort_pairs(pre, cam, tile)
    fl, got = _lists(it)
    assert fl[L.F_OVERFLOW] == 0 and int(fl[L.F_PAIRS]) == keys.shape[0]
    np.testing.assert_array_equal(got["keys"].view(np.uint64), keys)
    np.testing.assert_array_equal(got["recs"], vals.astype(np.int32))
    np.testing.assert_array_equal(got["ranges"].view(np.uint32), ranges)
    # generation indices and everything downstream as the per-tile binning
    ref = run_gpu(w.scene, [cam], tile=tile)
    _, want = _lists(ref)
    for k in want:
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    _same_iteration(it, ref, 1)


@pytest.mark.parametrize("tile,n", [((16, 16), 6000), ((8, 8), 300), ((16, 16), 20000)])
def test_radix_bin_long_tile_list(tile, n):
    """n pairs in one tile (the per-tile binning's long-list paths) and
    short lists elsewhere."""
    w = scenes.crowded_scene(1, n=n)
    cam = w.cameras[0]
    print(f"radix binning long list tile {tile} n {n}", flush=True)
    it = run_gpu(w.scene, [cam], tile=tile, flags=RADIX)
    pre = oracle.preprocess(w.scene, cam, tile)
    assert not (pre["near_edge"] != 0).any()
    keys, vals, ranges = oracle.sort_pairs(pre, cam, tile)
    fl, got = _lists(it)
    assert fl[L.F_OVERFLOW] == 0 and int(fl[L.F_PAIRS]) == keys.shape[0]
    r = ranges.reshape(-1, 2).astype(np.int64)
    assert (r[:, 1] - r[:, 0]).max() == n
    np.testing.assert_array_equal(got["keys"].view(np.uint64), keys)
    np.testing.assert_array_equal(got["recs"], vals.astype(np.int32))
    np.testing.assert_array_equal(got["ranges"].view(np.uint32), ranges)


def test_radix_bin_multi_view_iteration_equals_per_tile_binning():
    """Four views over 120k Gaussians, persistent splat-wise iteration with
    camera tangents: radix and per-tile binning bit for bit."""
    w = workload(4, n=120_000, n_views=4)
    gcs, gds = scenes.linear_loss_weights(47, w.cameras)
    print("radix binning, 4 views 120k: against the per-tile binning", flush=True)
    kw = dict(tile=(8, 8), lds=64, dL_dcolor=gcs, dL_ddepth=gds, pose=True)
    base = L.GS_PERSISTENT | L.GS_SPLAT_BWD
    a = run_gpu(w.scene, w.cameras, flags=base | RADIX, **kw)
    b = run_gpu(w.scene, w.cameras, flags=base, **kw)
    _, la = _lists(a)
    _, lb = _lists(b)
    for k in la:
        np.testing.assert_array_equal(la[k], lb[k], err_msg=k)
    _same_iteration(a, b, len(w.cameras))
    np.testing.assert_array_equal(a.dL_dpose.cpu().numpy(), b.dL_dpose.cpu().numpy())


@pytest.mark.parametrize("n,extra", [(300, 0), (3000, L.GS_SPLAT_BWD)])
def test_radix_bin_single_view_adam_iteration(n, extra):
    """The one-view iteration with Adam (its forward normally sorts the
    short lists; with the radix binning it only reads them): against the
    per-tile binning over two steps, parameters and moments bit for bit."""
    w = scenes.crowded_scene(3, n=n)
    cam = w.cameras[0]
    sc = w.scene
    print(f"radix binning, one-view Adam iteration n {n} flags {extra}", flush=True)
    rng = np.random.default_rng(12)
    tgt = t32(rng.uniform(0.0, 1.0, (3, cam.height, cam.width)).reshape(-1))
    cams = gsr.cameras_tensor([cam], DEV)

    def make(flags):
        g = gsr.Gaussians.from_scene(sc, DEV)
        cap = gsr.required_pairs(*g.tensors(), cams, [(cam.width, cam.height)], sc.sh_degree,
                                 (16, 16)) + 7
        plan = gsr.Plan(sc.n, sc.sh_degree, [(cam.width, cam.height)],
                        flags=L.GS_FUSED_L1 | extra | flags, pair_capacity=cap)
        return gsr.Iteration(plan, g, cams, target_rgb=tgt, adam_lrs=LRS)

    a, b = make(RADIX), make(0)
    for step in range(2):
        a.enqueue()
        b.enqueue()
        torch.cuda.synchronize()
        assert torch.equal(a.frame.color, b.frame.color), step
        assert torch.equal(a.frame.loss, b.frame.loss), step
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(a.g, f), getattr(b.g, f)), (step, f)
            assert torch.equal(getattr(a.m, f), getattr(b.m, f)), (step, f)
            assert torch.equal(getattr(a.v, f), getattr(b.v, f)), (step, f)


def test_radix_bin_graph_replay_equals_eager():
    w = workload(1)
    cam = w.cameras[0]
    tgt = t32(w.target_rgb[0].reshape(-1))
    flags = L.GS_FUSED_L1 | L.GS_SPLAT_BWD | RADIX

    def make():
        g = gsr.Gaussians.from_scene(w.scene, DEV)
        plan = gsr.Plan(w.scene.n, 0, [(cam.width, cam.height)], flags=flags,
                        pair_capacity=1 << 16)
        return gsr.Iteration(plan, g, gsr.cameras_tensor([cam], DEV), target_rgb=tgt,
                             adam_lrs=LRS)

    print("radix binning: graph replays against eager iterations", flush=True)
    eager, graphed = make(), make()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graphed.capture(s)
    for step in range(3):
        eager.enqueue()
        torch.cuda.synchronize()
        _ = (eager.frame.color * 2).sum().item()
        with torch.cuda.stream(s):
            graphed.replay(s)
        s.synchronize()
        for f in gsr.Gaussians.FIELDS:
            assert torch.equal(getattr(eager.g, f), getattr(graphed.g, f)), (step, f)
        assert torch.equal(eager.frame.color, graphed.frame.color)
        assert torch.equal(eager.frame.loss, graphed.frame.loss)
    assert int(graphed.step_dev.item()) == 3
    graphed.close()


def test_radix_bin_overflow_and_empty_inputs():
    w = workload(1)
    cam = w.cameras[0]
    print("radix binning: overflow, empty pool, view facing away", flush=True)
    it = run_gpu(w.scene, [cam], capacity=100, flags=RADIX)
    fl = it.plan.flags_of(it.ws)
    assert fl[L.F_OVERFLOW] == 1 and fl[L.F_PAIRS_WANTED] > 100 and fl[L.F_PAIRS] == 0
    col, dep, T, last = view_images(it, 0)
    assert (last == 0).all()
    empty = w.scene.subset(np.arange(0))
    it = run_gpu(empty, [cam], capacity=1, flags=RADIX)
    col, dep, T, last = view_images(it, 0)
    assert (col == 0).all() and (dep == 0).all() and (T == 1).all() and (last == 0).all()
    back = scenes.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                         np.diag([1.0, -1.0, -1.0]).astype(np.float32), np.zeros(3, np.float32),
                         bg=(0.1, 0.2, 0.3))
    gc, gd = scenes.linear_loss_weights(1, [back])
    it = run_gpu(w.scene, [back], capacity=1, dL_dcolor=gc, dL_ddepth=gd, flags=RADIX)
    col, _, _, _ = view_images(it, 0)
    np.testing.assert_allclose(col[0], 0.1, rtol=0, atol=1e-7)
    g = grads_np(it)
    assert all((g[f] == 0).all() for f in g)


def test_autotuner_searches_the_binning():
    """The autotuner times both binnings (and the other dimensions it is
    given) as captured graphs and returns the fastest, with its binning."""
    from paper_2410_00486_amd import tune
    w = workload(1)
    cam = w.cameras[0]
    tgt = t32(w.target_rgb[0].reshape(-1))
    g = gsr.Gaussians.from_scene(w.scene, DEV)
    print("autotuner over tiles / radix binning", flush=True)
    best, table = tune.autotune(g, gsr.cameras_tensor([cam], DEV), [(cam.width, cam.height)],
                                target_rgb=tgt, adam_lrs=LRS, tiles=[(16, 16)], lds_batches=[64],
                                chunks=[1], backwards=["splat"], binnings=["tiles", "radix"],
                                reps=2)
    assert sorted(r["binning"] for r in table) == ["radix", "tiles"]
    assert all(r["overflow"] == 0 and r["ms"] > 0 for r in table)
    assert best["binning"] in ("tiles", "radix") and best["ms"] == min(r["ms"] for r in table)
