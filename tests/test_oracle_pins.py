"""Pins of the FP64 oracle against facts it does not compute itself.

Every test here runs on the CPU.  Each one is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand, a wrong SH constant) fails at least one of them:

* rotation convention vs scipy's quaternion rotation matrices;
* SH basis (degrees 0-3, Condon-Shortley phase) vs scipy's complex SH;
* pinhole mean vs a homogeneous K[R|t] projection; EWA covariance vs a
  numerically differentiated projection; conic vs a matrix inverse;
* compositing closed forms (one isotropic Gaussian at the image centre, two
  stacked Gaussians, an opaque stack hitting the stop rule), the telescoping
  identity sum_k a_k T_k + T_final = 1, background for a transparent splat;
* the exact opacity-aware tile box vs sampled points on the a = 1/255 ellipse,
  and tiled == untiled rendering for every tile shape; the comparison-only
  3-sigma box vs numpy's eigenvalues and sampled points on its circle;
* invariances (rigid motion of scene + camera, q -> -q, isotropic => q-free);
* sort vs numpy's lexsort;
* the hand-derived backward vs FP64 central differences (all parameter
  groups, SH degrees 0 and 3, a clamped-Jacobian Gaussian, the stop rule)
  and the camera tangent vs finite differences of the perturbed pose;
* Adam vs torch.optim.Adam in float64; the L1 and opacity-regulariser
  gradients vs torch autograd.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from synth import scenes
from synth.scenes import Camera, Scene


def _cam(width=64, height=48, f=50.0, R=None, t=None, bg=(0.0, 0.0, 0.0), cx=None, cy=None):
    return Camera(width, height, f, f, width / 2.0 if cx is None else cx,
                  height / 2.0 if cy is None else cy,
                  np.eye(3) if R is None else np.asarray(R, np.float64),
                  np.zeros(3) if t is None else np.asarray(t, np.float64), 0.2, bg)


def _scene(means, log_scales, quats, logits, sh, deg=0):
    return Scene(np.asarray(means, np.float64).reshape(-1, 3),
                 np.asarray(log_scales, np.float64).reshape(-1, 3),
                 np.asarray(quats, np.float64).reshape(-1, 4),
                 np.asarray(logits, np.float64).reshape(-1),
                 np.asarray(sh, np.float64).reshape(-1, (deg + 1) ** 2, 3), deg)


def _dc_for_colour(c):
    # DC coefficient giving colour c for SH degree 0: c = sh0 * Y00 + 0.5
    return (np.asarray(c, np.float64) - 0.5) * 2.0 * math.sqrt(math.pi)


def _logit(o):
    return math.log(o / (1.0 - o))


# ---------------------------------------------------------------------------
# geometry pins
# ---------------------------------------------------------------------------

def test_rotation_convention_matches_scipy():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((50, 4)) * rng.uniform(0.3, 3.0, (50, 1))
    ls = rng.normal(-1.0, 0.5, (50, 3))
    cov = oracle.covariance3d(ls, q)
    for i in range(50):
        R = Rotation.from_quat([q[i, 1], q[i, 2], q[i, 3], q[i, 0]]).as_matrix()
        ref = R @ np.diag(np.exp(2 * ls[i])) @ R.T
        np.testing.assert_allclose(cov[i], ref, rtol=1e-12, atol=1e-14)


def _real_sh_scipy(l, m, d):
    """Real SH from scipy's complex SH (which carries the Condon-Shortley
    phase): sqrt(2) Im Y_l^|m| for m < 0, Y_l^0, sqrt(2) Re Y_l^m for m > 0."""
    theta = np.arccos(np.clip(d[2], -1, 1))
    phi = np.arctan2(d[1], d[0])
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    if m > 0:
        return math.sqrt(2.0) * sph_harm_y(l, m, theta, phi).real
    return math.sqrt(2.0) * sph_harm_y(l, -m, theta, phi).imag


def test_sh_basis_matches_scipy():
    """Colour of a Gaussian whose only SH coefficient is 0.1 on basis k is
    0.1 * Y_k(dir) + 0.5; dir is from a camera centre that is not the origin."""
    rng = np.random.default_rng(1)
    centre = np.array([0.3, -0.2, 0.1])
    n_dir = 12
    dirs = rng.standard_normal((n_dir, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dirs[:, 2] = np.abs(dirs[:, 2]) + 0.5          # in front of the camera
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    means, shs = [], []
    for k in range(16):
        for d in dirs:
            means.append(centre + 3.0 * d)
            sh = np.zeros((16, 3))
            sh[k, 0] = 0.1
            shs.append(sh)
    n = len(means)
    sc = _scene(means, np.full((n, 3), -3.0), np.tile([1.0, 0, 0, 0], (n, 1)), np.zeros(n),
                np.array(shs), deg=3)
    cam = _cam(200, 200, 20.0, t=-centre)
    pre = oracle.preprocess(sc, cam)
    lm = [(0, 0)] + [(1, m) for m in (-1, 0, 1)] + [(2, m) for m in range(-2, 3)] + \
         [(3, m) for m in range(-3, 4)]
    j = 0
    for k, (l, m) in enumerate(lm):
        for d in dirs:
            assert pre["status"][j] == 1
            ref = 0.1 * _real_sh_scipy(l, m, d) + 0.5
            assert abs(pre["rgb"][j, 0] - ref) < 1e-12, (k, l, m)
            j += 1


def test_mean2d_matches_homogeneous_projection():
    rng = np.random.default_rng(2)
    R, _ = scenes.random_pose(rng)
    t = np.array([0.1, -0.2, 0.3])
    cam = _cam(100, 80, 70.0, R=R, t=t, cx=47.0, cy=41.5)
    cam = dataclasses.replace(cam, fy=65.0)
    n = 30
    pts_cam = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(2, 5, n)], 1)
    means = (pts_cam - t) @ R                      # world points
    sc = _scene(means, np.full((n, 3), -2.5), np.tile([1.0, 0, 0, 0], (n, 1)), np.zeros(n),
                np.zeros((n, 1, 3)))
    pre = oracle.preprocess(sc, cam)
    K = np.array([[70.0, 0, 47.0], [0, 65.0, 41.5], [0, 0, 1]])
    P = K @ np.concatenate([R, t[:, None]], 1)
    h = (P @ np.concatenate([means, np.ones((n, 1))], 1).T).T
    ref = h[:, :2] / h[:, 2:3]
    vis = pre["status"] == 1
    assert vis.sum() > 20
    np.testing.assert_allclose(pre["mean2d"][vis], ref[vis], rtol=0, atol=1e-10)
    np.testing.assert_allclose(pre["depth"][vis], h[vis, 2], rtol=1e-13)


def test_ewa_covariance_matches_numerical_jacobian():
    """Sigma' = J W Sigma W^T J^T + 0.3 I with J the Jacobian of the pinhole
    map, here obtained by central differences (inside the FOV clamp)."""
    rng = np.random.default_rng(3)
    R, _ = scenes.random_pose(rng)
    t = np.array([0.05, 0.1, -0.1])
    cam = _cam(120, 90, 80.0, R=R, t=t)
    n = 25
    pts_cam = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 4, n)], 1)
    means = (pts_cam - t) @ R
    ls = rng.normal(-2.5, 0.4, (n, 3))
    q = rng.standard_normal((n, 4))
    sc = _scene(means, ls, q, np.full(n, 2.0), np.zeros((n, 1, 3)))
    pre = oracle.preprocess(sc, cam)

    def proj(tc):
        return np.array([80.0 * tc[0] / tc[2] + 60.0, 80.0 * tc[1] / tc[2] + 45.0])

    for i in range(n):
        assert pre["status"][i] == 1
        tc = R @ means[i] + t
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-6
            J[:, k] = (proj(tc + e) - proj(tc - e)) / 2e-6
        Rq = Rotation.from_quat([q[i, 1], q[i, 2], q[i, 3], q[i, 0]]).as_matrix()
        Sig = Rq @ np.diag(np.exp(2 * ls[i])) @ Rq.T
        ref = J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2)
        got = np.array([[pre["cov2d"][i, 0], pre["cov2d"][i, 1]], [pre["cov2d"][i, 1], pre["cov2d"][i, 2]]])
        np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-9)
        con = np.array([[pre["conic"][i, 0], pre["conic"][i, 1]], [pre["conic"][i, 1], pre["conic"][i, 2]]])
        np.testing.assert_allclose(con, np.linalg.inv(got), rtol=1e-12)


def test_tile_rect_covers_exact_alpha_ellipse():
    """The tile box must contain every point of the a = 1/255 ellipse
    (sampled), and the sampled extent must match the box half-widths."""
    rng = np.random.default_rng(4)
    n = 20
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 3, n)], 1)
    ls = rng.normal(-2.2, 0.5, (n, 3))
    logits = rng.normal(0.0, 1.5, n)
    sc = _scene(means, ls, rng.standard_normal((n, 4)), logits, np.zeros((n, 1, 3)))
    cam = _cam(160, 120, 100.0)
    for tile in [(16, 16), (8, 8), (16, 8)]:
        pre = oracle.preprocess(sc, cam, tile)
        for i in range(n):
            if pre["status"][i] != 1:
                continue
            A, B, C = pre["cov2d"][i]
            L = np.linalg.cholesky(np.array([[A, B], [B, C]]))
            kappa = math.sqrt(2 * math.log(255 * pre["opacity"][i]))
            ang = np.linspace(0, 2 * np.pi, 40001)
            pts = pre["mean2d"][i][:, None] + kappa * L @ np.stack([np.cos(ang), np.sin(ang)])
            # on the boundary alpha = o exp(-kappa^2/2) = 1/255 by construction of L;
            # the sampled extent approaches the box half-width from below
            for ax, var in ((0, A), (1, C)):
                ext = kappa * math.sqrt(var)
                got = pts[ax].max() - pre["mean2d"][i, ax]
                assert ext * (1 - 1e-7) <= got <= ext * (1 + 1e-12)
            x0, y0, x1, y1 = pre["rect"][i]
            inside = (pts[0] >= 0) & (pts[0] < 160) & (pts[1] >= 0) & (pts[1] < 120)
            tx, ty = np.floor(pts[0][inside] / tile[0]), np.floor(pts[1][inside] / tile[1])
            assert np.all((tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1))


def test_three_sigma_box_pins():
    """The comparison-only 3-sigma tile box: the square of half-width
    3 sqrt(lambda_max) of the projected covariance (lambda_max from numpy's
    symmetric eigensolver), padded by the same margin as the exact box.  The
    box must hold every sampled point of the 3-sigma circle, equal the tile
    range of that square wherever the eigenvalue gap is not floored (the
    floor only widens nearly isotropic boxes), and leave the projection, the
    culling of invisible Gaussians and the compositing rules as they are: a
    3-sigma render whose single tile is the whole image equals the brute
    force over the same records."""
    rng = np.random.default_rng(21)
    n = 60
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.45, 0.45, n), rng.uniform(2, 3.5, n)], 1)
    ls = rng.normal(-2.5, 0.6, (n, 3))
    logits = rng.normal(0.0, 1.5, n)
    sc = _scene(means, ls, rng.standard_normal((n, 4)), logits, _dc_for_colour(rng.uniform(0, 1, (n, 1, 3))))
    cam = _cam(160, 120, 100.0)
    checked_eq = 0
    for tile in [(16, 16), (8, 8), (16, 8)]:
        pre = oracle.preprocess(sc, cam, tile, cutoff="3sigma")
        ex = oracle.preprocess(sc, cam, tile)
        np.testing.assert_array_equal(pre["mean2d"], ex["mean2d"])
        np.testing.assert_array_equal(pre["conic"], ex["conic"])
        tx_n, ty_n = (160 + tile[0] - 1) // tile[0], (120 + tile[1] - 1) // tile[1]
        for i in range(n):
            if pre["status"][i] != 1:
                continue
            A, B, C = pre["cov2d"][i]
            lam = np.linalg.eigvalsh(np.array([[A, B], [B, C]]))
            r = 3.0 * math.sqrt(lam[1])
            ang = np.linspace(0, 2 * np.pi, 4001)
            pts = pre["mean2d"][i][:, None] + r * np.stack([np.cos(ang), np.sin(ang)])
            x0, y0, x1, y1 = pre["rect"][i]
            inside = (pts[0] >= 0) & (pts[0] < 160) & (pts[1] >= 0) & (pts[1] < 120)
            tx, ty = np.floor(pts[0][inside] / tile[0]), np.floor(pts[1][inside] / tile[1])
            assert np.all((tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1))
            gap = 0.5 * (lam[1] - lam[0])
            if gap * gap < 0.1 * (1 + 1e-9):
                continue
            h = r * (1 + 1e-4) + 1e-3
            mx, my = pre["mean2d"][i]
            lo = np.array([(mx - h) / tile[0], (my - h) / tile[1]])
            hi = np.array([(mx + h) / tile[0], (my + h) / tile[1]])
            if np.any(np.abs(np.concatenate([lo, hi]) - np.round(np.concatenate([lo, hi]))) < 1e-9):
                continue
            want = [int(np.clip(np.floor(lo[0]), 0, tx_n)), int(np.clip(np.floor(lo[1]), 0, ty_n)),
                    int(np.clip(np.floor(hi[0]) + 1, 0, tx_n)), int(np.clip(np.floor(hi[1]) + 1, 0, ty_n))]
            assert list(pre["rect"][i]) == want, (i, tile, list(pre["rect"][i]), want)
            checked_eq += 1
    assert checked_eq > 30
    whole = oracle.preprocess(sc, cam, (160, 120), cutoff="3sigma")
    tiled = oracle.render(sc, cam, (160, 120), cutoff="3sigma", pre=whole)
    brute = oracle.render_untiled(sc, cam, pre=whole)
    np.testing.assert_array_equal(tiled["color"], brute["color"])
    np.testing.assert_array_equal(tiled["depth"], brute["depth"])


# ---------------------------------------------------------------------------
# compositing closed forms
# ---------------------------------------------------------------------------

def _alpha_iso(o, f, s, z, dx, dy):
    var = (f * s / z) ** 2 + 0.3
    oG = o * math.exp(-(dx * dx + dy * dy) / (2 * var))
    a = min(0.99, oG)
    return a if a >= 1 / 255 else 0.0


def test_single_isotropic_gaussian_closed_form():
    f, s, z, o, c = 50.0, 0.04, 2.5, 0.8, np.array([0.9, 0.4, 0.2])
    sc = _scene([0, 0, z], [math.log(s)] * 3, [0.3, -0.5, 0.2, 0.7], [_logit(o)],
                _dc_for_colour(c)[None, :])
    cam = _cam(64, 48, f)
    out = oracle.render(sc, cam)
    pre = out["pre"]
    var = (f * s / z) ** 2 + 0.3
    np.testing.assert_allclose(pre["cov2d"][0], [var, 0, var], atol=1e-12)
    np.testing.assert_allclose(pre["conic"][0], [1 / var, 0, 1 / var], atol=1e-12)
    np.testing.assert_allclose(pre["mean2d"][0], [32, 24], atol=1e-12)
    for py in range(48):
        for px in range(64):
            a = _alpha_iso(o, f, s, z, 32 - (px + 0.5), 24 - (py + 0.5))
            assert abs(out["color"][0, py, px] - c[0] * a) < 1e-12
            assert abs(out["color"][2, py, px] - c[2] * a) < 1e-12
            assert abs(out["depth"][py, px] - z * a) < 1e-12
            assert abs(out["T_final"][py, px] - (1 - a)) < 1e-12
    # four-fold symmetry about the image centre (a pixel corner)
    col = out["color"][0]
    np.testing.assert_array_equal(col, col[::-1, :])
    np.testing.assert_array_equal(col, col[:, ::-1])


def test_two_stacked_gaussians_closed_form():
    f = 50.0
    o1, o2 = 0.6, 0.7
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.5])
    z1, z2 = 2.0, 3.0
    s1, s2 = 0.05, 0.075                    # same footprint: s/z equal
    sc = _scene([[0, 0, z2], [0, 0, z1]], [[math.log(s2)] * 3, [math.log(s1)] * 3],
                [[1, 0, 0, 0], [1, 0, 0, 0]], [_logit(o2), _logit(o1)],
                np.stack([_dc_for_colour(c2), _dc_for_colour(c1)])[:, None, :])
    out = oracle.render(sc, _cam(64, 48, f))
    for (px, py) in [(31, 23), (32, 24), (28, 20), (35, 27)]:
        a1 = _alpha_iso(o1, f, s1, z1, 32 - (px + 0.5), 24 - (py + 0.5))
        a2 = _alpha_iso(o2, f, s2, z2, 32 - (px + 0.5), 24 - (py + 0.5))
        ref = c1 * a1 + c2 * a2 * (1 - a1)
        np.testing.assert_allclose(out["color"][:, py, px], ref, atol=1e-12)
        assert abs(out["depth"][py, px] - (z1 * a1 + z2 * a2 * (1 - a1))) < 1e-12
        assert abs(out["T_final"][py, px] - (1 - a1) * (1 - a2)) < 1e-12
    # swapping the depths swaps the blend order
    sc2 = _scene([[0, 0, z1], [0, 0, z2]], [[math.log(s1)] * 3, [math.log(s2)] * 3],
                 [[1, 0, 0, 0], [1, 0, 0, 0]], [_logit(o2), _logit(o1)],
                 np.stack([_dc_for_colour(c2), _dc_for_colour(c1)])[:, None, :])
    out2 = oracle.render(sc2, _cam(64, 48, f))
    px, py = 32, 24
    a_front = _alpha_iso(o2, f, s1, z1, -0.5, -0.5)
    a_back = _alpha_iso(o1, f, s2, z2, -0.5, -0.5)
    ref = c2 * a_front + c1 * a_back * (1 - a_front)
    np.testing.assert_allclose(out2["color"][:, py, px], ref, atol=1e-12)


def test_stop_rule_closed_form():
    """An opaque stack with a = 0.95 at the centre: T goes 1, .05, .0025,
    .000125; the fourth would take T below 1e-4, so it is not blended."""
    n = 6
    f, z0 = 50.0, 2.0
    zs = z0 + 0.1 * np.arange(n)
    s = 0.5 * zs / f * 10                   # large footprint, same for all
    o = 0.95 / math.exp(-(0.5 ** 2 + 0.5 ** 2) / (2 * ((f * s[0] / zs[0]) ** 2 + 0.3)))
    sc = _scene(np.stack([np.zeros(n), np.zeros(n), zs], 1), np.log(s)[:, None].repeat(3, 1),
                np.tile([1.0, 0, 0, 0], (n, 1)), np.full(n, _logit(o)),
                np.tile(_dc_for_colour([1.0, 0.5, 0.0]), (n, 1))[:, None, :])
    out = oracle.render(sc, _cam(64, 48, f))
    px, py = 32, 24
    assert out["last"][py, px] == 3
    assert abs(out["T_final"][py, px] - 0.05 ** 3) < 1e-12
    ref = sum(0.95 * 0.05 ** k for k in range(3))
    assert abs(out["color"][0, py, px] - ref) < 1e-12
    assert out["T_final"].min() >= 1e-4


def test_weights_telescope_to_one():
    """With every colour 1 and a black background, C = sum_k a_k T_k, so
    C + T_final = 1 exactly (up to rounding) at every pixel."""
    w = scenes.slab_128x96(seed=77, n=600)
    sc = w.scene.copy()
    sc.sh = np.tile(_dc_for_colour([1.0, 1.0, 1.0]), (sc.n, 1))[:, None, :]
    out = oracle.render(sc, w.cameras[0])
    np.testing.assert_allclose(out["color"][0] + out["T_final"], 1.0, atol=1e-12)
    assert out["last"].max() > 5 and out["T_final"].min() < 0.05


def test_transparent_gaussian_shows_background():
    bg = (0.2, 0.3, 0.4)
    sc = _scene([0, 0, 2.0], [-2.0] * 3, [1, 0, 0, 0], [_logit(0.003)],
                _dc_for_colour([1, 1, 1])[None, None, :])
    out = oracle.render(sc, _cam(32, 24, 30.0, bg=bg))
    assert out["pre"]["status"][0] == 0
    for ch in range(3):
        np.testing.assert_allclose(out["color"][ch], bg[ch], atol=0)
    np.testing.assert_array_equal(out["T_final"], 1.0)


# ---------------------------------------------------------------------------
# invariances and tiling
# ---------------------------------------------------------------------------

def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def test_rigid_motion_invariance():
    w = scenes.slab_128x96(seed=5, n=400)
    sc = w.scene.copy()
    sc = _scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)
    cam = _cam(128, 96, 100.0)
    base = oracle.render(sc, cam)
    rng = np.random.default_rng(6)
    rot = Rotation.from_rotvec(rng.normal(0, 0.7, 3))
    Q = rot.as_matrix()
    xyzw = rot.as_quat()
    qQ = np.array([xyzw[3], xyzw[0], xyzw[1], xyzw[2]])
    d = rng.normal(0, 1.0, 3)
    moved = _scene(sc.means @ Q.T + d, sc.log_scales, _quat_mul(qQ, sc.quats), sc.opacity_logits, sc.sh)
    cam2 = _cam(128, 96, 100.0, R=Q.T, t=-Q.T @ d)
    out = oracle.render(moved, cam2)
    ok = (base["flag"] == 0) & (out["flag"] == 0)
    assert ok.mean() > 0.999
    np.testing.assert_allclose(out["color"][:, ok], base["color"][:, ok], atol=1e-9)
    np.testing.assert_allclose(out["depth"][ok], base["depth"][ok], atol=1e-9)


def test_quaternion_sign_and_isotropic_invariance():
    w = scenes.slab_128x96(seed=8, n=300)
    sc = _scene(w.scene.means, w.scene.log_scales, w.scene.quats, w.scene.opacity_logits, w.scene.sh)
    cam = _cam(128, 96, 100.0)
    base = oracle.render(sc, cam)
    neg = _scene(sc.means, sc.log_scales, -sc.quats, sc.opacity_logits, sc.sh)
    out = oracle.render(neg, cam)
    np.testing.assert_array_equal(out["color"], base["color"])
    iso_ls = np.repeat(sc.log_scales[:, :1], 3, axis=1)
    a = oracle.render(_scene(sc.means, iso_ls, sc.quats, sc.opacity_logits, sc.sh), cam)
    b = oracle.render(_scene(sc.means, iso_ls, np.tile([1.0, 0, 0, 0], (sc.n, 1)),
                             sc.opacity_logits, sc.sh), cam)
    np.testing.assert_allclose(a["color"], b["color"], atol=1e-12)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8)])
def test_tiled_equals_untiled(tile):
    w = scenes.slab_128x96(seed=9, n=800)
    cam = w.cameras[0]
    tiled = oracle.render(w.scene, cam, tile)
    brute = oracle.render_untiled(w.scene, cam)
    np.testing.assert_array_equal(tiled["color"], brute["color"])
    np.testing.assert_array_equal(tiled["depth"], brute["depth"])
    np.testing.assert_array_equal(tiled["T_final"], brute["T_final"])


def test_sort_matches_lexsort():
    w = scenes.slab_128x96(seed=10, n=1500)
    cam = w.cameras[0]
    pre = oracle.preprocess(w.scene, cam)
    keys, vals, ranges = oracle.sort_pairs(pre, cam)
    # brute force: enumerate pairs, order by (tile, depth bits, index)
    tiles, dbits, idx = [], [], []
    tx = (cam.width + 15) // 16
    for i in np.nonzero(pre["status"] == 1)[0]:
        x0, y0, x1, y1 = pre["rect"][i]
        for y in range(y0, y1):
            for x in range(x0, x1):
                tiles.append(y * tx + x)
                dbits.append(pre["depth32"][i:i + 1].view(np.uint32)[0])
                idx.append(i)
    tiles, dbits, idx = map(np.array, (tiles, dbits, idx))
    order = np.lexsort((idx, dbits, tiles))
    ref_keys = (tiles[order].astype(np.uint64) << np.uint64(32)) | dbits[order].astype(np.uint64)
    np.testing.assert_array_equal(keys, ref_keys)
    np.testing.assert_array_equal(vals, idx[order])
    for t in range(ranges.shape[0] // 2):
        sel = np.nonzero(tiles[order] == t)[0]
        if sel.size:
            assert ranges[2 * t] == sel[0] and ranges[2 * t + 1] == sel[-1] + 1
        else:
            assert ranges[2 * t] == ranges[2 * t + 1]


# ---------------------------------------------------------------------------
# backward: FP64 finite differences
# ---------------------------------------------------------------------------

def _loss(sc, cams, gC, gD):
    fw = [oracle.render(sc, c) for c in cams]
    return oracle.linear_loss(fw, gC, gD), fw


def _fd_check(sc, cams, gC, gD, groups=("means", "log_scales", "quats", "opacity_logits", "sh")):
    L0, fw = _loss(sc, cams, gC, gD)
    for f in fw:
        assert f["flag"].sum() == 0, "scene has a decision inside the band; pick another seed"
    grads, _ = oracle.backward(sc, cams, gC, gD)
    for name in groups:
        arr = getattr(sc, name)
        an = grads[name].reshape(-1)
        flat = arr.reshape(-1)
        scale = np.abs(an).max()
        assert scale > 0, name
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            Lp, _ = _loss(sc, cams, gC, gD)
            flat[j] = old - h
            Lm, _ = _loss(sc, cams, gC, gD)
            flat[j] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - an[j]) <= 1e-6 * abs(an[j]) + 2e-7 * scale, (name, j, fd, an[j])


def _as64(sc):
    return _scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, sc.sh_degree)


@pytest.mark.parametrize("seed,deg", [(11, 0), (12, 3)])
def test_backward_matches_finite_differences(seed, deg):
    w = scenes.tiny_scene(seed, n=8, degree=deg)
    sc = _as64(w.scene)
    gC, gD = scenes.linear_loss_weights(seed + 100, w.cameras)
    gC = [g * 100 for g in gC]
    gD = [g * 100 for g in gD]
    _fd_check(sc, w.cameras, gC, gD)


def test_backward_fd_dense_stack_hits_stop_rule():
    """Many overlapping opaque Gaussians so that T reaches the 1e-4 stop."""
    rng = np.random.default_rng(13)
    n = 14
    means = np.stack([rng.uniform(-0.15, 0.15, n), rng.uniform(-0.1, 0.1, n), rng.uniform(2, 3, n)], 1)
    sc = _scene(means, rng.normal(-1.6, 0.15, (n, 3)), rng.standard_normal((n, 4)),
                rng.normal(3.0, 0.5, n), rng.uniform(-1, 1, (n, 1, 3)))
    cam = _cam(24, 20, 30.0)
    out = oracle.render(sc, cam)
    assert (out["last"] < out["pre"]["tiles_touched"].sum()).any()
    assert out["T_final"].min() < 2e-3
    gC, gD = scenes.linear_loss_weights(14, [cam])
    _fd_check(sc, [cam], [g * 100 for g in gC], [g * 100 for g in gD],
              groups=("means", "log_scales", "opacity_logits"))


def test_backward_fd_clamped_jacobian():
    """A large Gaussian whose centre lies beyond 1.3x the half FOV (clamped
    Jacobian) but whose footprint reaches into the image."""
    sc = _scene([[2.2, 0.1, 2.0], [0.0, 0.0, 2.5]], [[-0.4, -0.9, -0.6], [-2.0, -2.2, -2.1]],
                [[0.9, 0.2, -0.3, 0.1], [0.5, 0.1, 0.4, -0.2]], [1.5, 0.5],
                np.array([_dc_for_colour([0.8, 0.3, 0.6]), _dc_for_colour([0.2, 0.7, 0.4])])[:, None, :])
    cam = _cam(32, 24, 30.0)
    pre = oracle.preprocess(sc, cam)
    assert pre["status"][0] == 1 and pre["mean2d"][0, 0] > 16 + 1.3 * 16
    gC, gD = scenes.linear_loss_weights(15, [cam])
    _fd_check(sc, [cam], [g * 100 for g in gC], [g * 100 for g in gD],
              groups=("means", "log_scales", "quats"))


def test_pose_gradient_matches_finite_differences():
    w = scenes.tiny_scene(16, n=10, degree=3)
    sc = _as64(w.scene)
    rng = np.random.default_rng(17)
    R, t = scenes.random_pose(rng, 0.05, 0.05)
    cam = _cam(32, 24, 30.0, R=R, t=t)
    gC, gD = scenes.linear_loss_weights(18, [cam])
    gC, gD = [gC[0] * 100], [gD[0] * 100]
    _, pose = oracle.backward(sc, [cam], gC, gD)
    pose = pose[0]
    for k in range(6):
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            xi = np.zeros(6); xi[k] = sgn * h
            Rp = Rotation.from_rotvec(xi[3:]).as_matrix()
            c2 = _cam(32, 24, 30.0, R=Rp @ R, t=Rp @ t + xi[:3])
            f = oracle.render(sc, c2)
            vals.append(oracle.linear_loss([f], gC, gD))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - pose[k]) <= 1e-6 * abs(pose[k]) + 1e-7 * np.abs(pose).max(), (k, fd, pose[k])


def test_pose_tangent_away_from_zero_matches_finite_differences():
    """The gradient of the tangent xi at xi != 0 (the autograd path renders at
    the retracted pose R' = Exp(phi) R, t' = Exp(phi) t + rho): the camera
    gradient at the retracted pose pulled back through the SO(3) left
    Jacobian, against FP64 central differences of the loss over xi (the
    rotation from scipy's rotvec map)."""
    w = scenes.tiny_scene(16, n=10, degree=3)
    sc = _as64(w.scene)
    rng = np.random.default_rng(17)
    R, t = scenes.random_pose(rng, 0.05, 0.05)
    cam = _cam(32, 24, 30.0, R=R, t=t)
    gC, gD = scenes.linear_loss_weights(18, [cam])
    gC, gD = [gC[0] * 100], [gD[0] * 100]
    xi = np.array([0.03, -0.02, 0.025, 0.04, -0.05, 0.03])
    cx = oracle.retract_camera(cam, xi, round32=False)
    _, g_delta = oracle.backward(sc, [cx], gC, gD)
    g_xi = oracle.pose_tangent_vjp(xi, g_delta)[0]
    assert np.linalg.norm(g_xi[3:] - g_delta[0, 3:]) > 1e-3 * np.linalg.norm(g_xi)  # not the identity here
    for k in range(6):
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            x2 = xi.copy()
            x2[k] += sgn * h
            f = oracle.render(sc, oracle.retract_camera(cam, x2, round32=False))
            vals.append(oracle.linear_loss([f], gC, gD))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g_xi[k]) <= 1e-6 * abs(g_xi[k]) + 1e-7 * np.abs(g_xi).max(), (k, fd, g_xi[k])


def test_so3_left_jacobian_series():
    """J from its power series against the closed form I + (1-cos)/th^2 K +
    (th - sin)/th^3 K^2 and against Exp(phi + eps e_k) Exp(phi)^T = Exp(eps J e_k)."""
    phi = np.array([0.3, -0.7, 0.4])
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    closed = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K
    J = oracle.so3_left_jacobian(phi)
    np.testing.assert_allclose(J, closed, atol=1e-14)
    for k in range(3):
        e = np.zeros(3); e[k] = 1e-6
        D = Rotation.from_matrix(oracle.so3_exp(phi + e) @ oracle.so3_exp(phi).T).as_rotvec()
        Dm = Rotation.from_matrix(oracle.so3_exp(phi - e) @ oracle.so3_exp(phi).T).as_rotvec()
        np.testing.assert_allclose((D - Dm) / 2e-6, J[:, k], atol=1e-8)
    assert np.allclose(oracle.so3_left_jacobian(np.zeros(3)), np.eye(3))


def test_pose_translation_equals_summed_mean_gradient():
    """Translating the camera by rho equals moving every mean by W^T rho, so
    g_rho = W sum_i g_p,i."""
    w = scenes.slab_128x96(seed=19, n=500)
    rng = np.random.default_rng(20)
    R, t = scenes.random_pose(rng, 0.1, 0.1)
    cam = dataclasses.replace(w.cameras[0], R=R, t=t)
    sc = _as64(w.scene)
    gC, gD = scenes.linear_loss_weights(21, [cam])
    grads, pose = oracle.backward(sc, [cam], gC, gD)
    np.testing.assert_allclose(pose[0, :3], R @ grads["means"].sum(0), rtol=1e-9,
                               atol=1e-12 * np.abs(pose).max())


def test_isotropic_gaussians_have_zero_quaternion_gradient():
    w = scenes.tiny_scene(22, n=8, degree=0)
    sc = _as64(w.scene)
    sc.log_scales = np.repeat(sc.log_scales[:, :1], 3, axis=1)
    gC, gD = scenes.linear_loss_weights(23, w.cameras)
    grads, _ = oracle.backward(sc, w.cameras, gC, gD)
    assert np.abs(grads["means"]).max() > 0
    assert np.abs(grads["quats"]).max() < 1e-12 * np.abs(grads["log_scales"]).max()


# ---------------------------------------------------------------------------
# loss and optimiser
# ---------------------------------------------------------------------------

def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(24)
    p0 = rng.standard_normal(1000)
    p = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-15, foreach=False)
    mine, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    for step in range(1, 6):
        g = rng.standard_normal(1000)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        mine, m, v = oracle.adam_step(mine, g, m, v, step, 3e-3, 0.9, 0.999, 1e-15)
    np.testing.assert_allclose(mine, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_l1_and_opacity_regulariser_grads_match_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(25)
    C = rng.uniform(0, 1, (3, 6, 7)); Ct = rng.uniform(0, 1, (3, 6, 7))
    D = rng.uniform(1, 3, (6, 7)); Dt = rng.uniform(1, 3, (6, 7))
    Ct[0, 0, 0] = C[0, 0, 0]                   # a zero residual: sign(0) = 0
    loss, gC, gD = oracle.l1_loss_and_grads(C, D, Ct, Dt, 0.1)
    tc = torch.tensor(C, requires_grad=True); td = torch.tensor(D, requires_grad=True)
    ref = (tc - torch.tensor(Ct)).abs().mean() + 0.1 * (td - torch.tensor(Dt)).abs().mean()
    ref.backward()
    assert abs(loss - ref.item()) < 1e-14
    np.testing.assert_allclose(gC, tc.grad.numpy(), atol=1e-15)
    np.testing.assert_allclose(gD, td.grad.numpy(), atol=1e-15)
    x = rng.normal(0, 2, 50)
    tx = torch.tensor(x, requires_grad=True)
    (0.001 * torch.sigmoid(tx).abs().mean()).backward()
    np.testing.assert_allclose(oracle.opacity_reg_grad(x, 0.001), tx.grad.numpy(), rtol=1e-12)


def test_near_threshold_pixels_are_flagged():
    """A Gaussian whose peak alpha sits exactly at 1/255 at a pixel centre
    makes that pixel a flagged (near-decision) pixel."""
    f, s, z = 30.0, 0.05, 2.0
    var = (f * s / z) ** 2 + 0.3
    G = math.exp(-(0.5 ** 2 + 0.5 ** 2) / (2 * var))
    o = (1 / 255) / G
    sc = _scene([0, 0, z], [math.log(s)] * 3, [1, 0, 0, 0], [_logit(o)],
                _dc_for_colour([1, 1, 1])[None, None, :])
    out = oracle.render(sc, _cam(32, 24, f))
    assert out["flag"][12, 16] == 1 and out["flag"][11, 15] == 1
    assert out["flag"].sum() == 4
