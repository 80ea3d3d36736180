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


def oracle_reference(scene, cams, gcs, gds, tile=(16, 16), alt_gcs=None, alt_gds=None):
    """Oracle gradients summed over the views, the per-view camera tangents,
    and the Gaussians excluded from the strict gradient check.

    A Gaussian is excluded when (a) one of its own decisions (the 0.99 clamp,
    the 1/255 skip, the 1e-4 stop) lies within a relative 1e-5 of its
    threshold at some pixel, or its tile-box edge or depth rounding is
    ambiguous; or (b) its oracle gradient moves by more than a quarter of its
    tolerance when every such near-threshold decision takes the other branch
    (the oracle's flip_band mode) and, if given, the upstream gradients are
    replaced by alt_gcs / alt_gds (the L1 signs undecided at FP32 accuracy).
    Everything else is checked strictly.  Returns (grads, poses, exclude,
    poses_flipped)."""
    cams = list(cams)
    grads, poses = oracle.backward(scene, cams, gcs, gds, tile)
    alt_gcs = gcs if alt_gcs is None else alt_gcs
    alt_gds = gds if alt_gds is None else alt_gds
    flipped, poses_f = oracle.backward(scene, cams, alt_gcs, alt_gds, tile, flip_band=True)
    n = scene.n
    exclude = np.zeros(n, bool)
    for f in grads:
        a = grads[f].reshape(n, -1)
        b = flipped[f].reshape(n, -1)
        rms = float(np.sqrt(np.mean(a * a))) if a.size else 0.0
        tol = GRAD_RTOL * np.abs(a) + GRAD_ATOL_RMS * rms
        exclude |= (np.abs(a - b) > 0.25 * tol).any(axis=1)
    for cam in cams:
        ref = oracle.render(scene, cam, tile)
        pre = ref["pre"]
        exclude |= (pre["status"] == 1) & (pre["near_edge"] != 0)
        _, g, kind = oracle.flag_decisions(ref, cam, tile)
        exclude[g[kind < 8]] = True
    return grads, poses, exclude, poses_f


def decided_target(rendered, target, margin=1e-4):
    """`target` with every residual against the oracle's render `rendered`
    pushed out to at least `margin` (same sign, zero counted as positive):
    the L1 sign of every pixel is then decided at FP32 accuracy, since the
    GPU image is within 1e-5 relative (in practice 1e-6) of the oracle's."""
    rendered = np.asarray(rendered, np.float64)
    target = np.asarray(target, np.float64)
    r = target - rendered
    sgn = np.where(r >= 0.0, 1.0, -1.0)
    out = np.where(np.abs(r) < margin, rendered + sgn * margin, target).astype(np.float32)
    assert (np.abs(out.astype(np.float64) - rendered) >= 0.9 * margin).all()
    return out


def visible_count(scene, cams, tile=(16, 16)):
    """Gaussians visible (non-empty tile box) in at least one view."""
    vis = np.zeros(scene.n, bool)
    for cam in cams:
        vis |= oracle.preprocess(scene, cam, tile)["status"] == 1
    return int(vis.sum())


def assert_pose_close(got, ref, ref_flipped=None, rtol=1e-3):
    """Camera tangents per view within rtol in norm.  A camera tangent sums
    over every blended pair of the view, so no Gaussian can be left out of
    it: instead its allowance grows by its sensitivity to the decisions taken
    within a relative 1e-5 of their thresholds (the oracle's flip-band
    result, whose distance from the plain one must itself stay below rtol;
    FP32 may take either branch of those decisions)."""
    got = np.asarray(got, np.float64).reshape(-1, 6)
    ref = np.asarray(ref, np.float64).reshape(-1, 6)
    for v in range(ref.shape[0]):
        nr = np.linalg.norm(ref[v])
        sens = 0.0
        if ref_flipped is not None:
            sens = float(np.linalg.norm(np.asarray(ref_flipped, np.float64).reshape(-1, 6)[v] - ref[v]))
            assert sens <= rtol * nr, (v, sens / nr)
        assert np.linalg.norm(got[v] - ref[v]) <= rtol * nr + sens, (v, got[v], ref[v])


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


def assert_grads_close(got: dict, ref: dict, exclude=None, fields=gsr.Gaussians.FIELDS,
                       visible=None, max_excluded=0.01):
    """Element-wise and norm check of the gradients; with `visible` (the
    number of visible Gaussians) the excluded ones must be fewer than
    max_excluded of them."""
    report = {}
    if exclude is not None and visible is not None:
        assert int(exclude.sum()) <= max(2, max_excluded * visible), (
            f"{int(exclude.sum())} of {visible} visible Gaussians excluded")
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


def view_tile_offsets(cams, tile):
    """First global tile id of each view (tiles numbered view by view)."""
    offs, t = [], 0
    for c in cams:
        offs.append(t)
        t += ((c.width + tile[0] - 1) // tile[0]) * ((c.height + tile[1] - 1) // tile[1])
    return offs


def assert_sorted_lists_match_oracle(it, scene, cams, tile, views):
    """The binned, depth-sorted pair lists of `views` against the oracle's
    stable sort, bit for bit: keys (global tile << 32 | float32 depth bits)
    and record ids.  Pairs of Gaussians whose tile-box edge is ambiguous
    (within a relative 1e-9 of a tile boundary) are dropped from both sides
    first: their extra or missing edge tile holds no pixel they blend.  The
    ranges must delimit the device keys' tiles."""
    plan, ws = it.plan, it.ws
    fl = plan.flags_of(ws)
    assert fl[L.F_OVERFLOW] == 0
    P = int(fl[L.F_PAIRS])
    T = plan.total_tiles
    gk = plan.region(ws, L.GS_WS_SORTED_KEYS, torch.int64, P).cpu().numpy().view(np.uint64)
    gr = plan.region(ws, L.GS_WS_SORTED_RECS, torch.int32, P).cpu().numpy().astype(np.int64)
    grg = plan.region(ws, L.GS_WS_RANGES, torch.int32, 2 * T).cpu().numpy().view(np.uint32)
    grg = grg.reshape(T, 2).astype(np.int64)
    # ranges delimit the tiles of the device keys
    tiles = (gk >> np.uint64(32)).astype(np.int64)
    assert (np.diff(tiles) >= 0).all()
    cnt = np.bincount(tiles, minlength=T)
    np.testing.assert_array_equal(grg[:, 1] - grg[:, 0], cnt)
    nz = cnt > 0
    np.testing.assert_array_equal(grg[nz, 0], np.searchsorted(tiles, np.nonzero(nz)[0]))
    offs = view_tile_offsets(cams, tile)
    n = scene.n
    for v in views:
        pre = oracle.preprocess(scene, cams[v], tile)
        keys, vals, _ = oracle.sort_pairs(pre, cams[v], tile)
        edge = np.nonzero((pre["status"] == 1) & (pre["near_edge"] != 0))[0]
        ok_o = ~np.isin(vals.astype(np.int64), edge)
        lo = offs[v]
        hi = offs[v + 1] if v + 1 < len(offs) else T
        mine = (tiles >= lo) & (tiles < hi)
        ok_g = mine & ~np.isin(gr - v * n, edge)
        np.testing.assert_array_equal(gk[ok_g], keys[ok_o] + (np.uint64(lo) << np.uint64(32)))
        np.testing.assert_array_equal(gr[ok_g] - v * n, vals[ok_o].astype(np.int64))
