"""Seeded synthetic inputs for the rasterizer and its oracle.

This module is the only code shared by the HIP path and the FP64 oracle.  It
draws scenes, cameras, targets and upstream gradients from numpy's PCG64
generator and holds none of the rendering method's arithmetic: no projection,
no compositing, no gradients.  Every array leaves here as float32 (the
parameters the GPU optimises); the oracle upcasts the same arrays to float64.

Workloads (sizes and distributions follow the indoor RGB-D mapping setting of
CaRtGS, Sec. IV-A; the datasets themselves are not used or reproduced):

* ``slab_128x96`` -- 128x96 pinhole, 2,000 Gaussians in a slab in front of an
  identity camera, SH degree 0, random target image.
* ``room_1200x680`` -- 1200x680 view inside a 6x5x3 m box room with 20 boxes,
  300k Gaussians seeded on the surfaces, SH degree 3.
* ``room_640x480_pose`` -- 640x480 view of a 150k-Gaussian room, pose perturbed from
  the ground truth for the camera-gradient check.
* ``keyframes8_mixed`` -- 8 keyframes of mixed resolution over a shared 500k pool.
* ``keyframes16_1200x680`` -- 16 keyframes at 1200x680 over a 2M-Gaussian four-room
  layout with 30% near-transparent Gaussians.

Conventions: world z is up; cameras look along their +z axis with +x right
and +y down; a camera stores the world->camera rotation ``R`` (row-major) and
translation ``t`` so that x_cam = R x_world + t.  Quaternions are (w, x, y, z)
and unnormalised; scales are log-scales; opacities are logits; SH
coefficients are laid out [N][(deg+1)^2][3].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Real SH band-0 basis value 1/(2*sqrt(pi)); used only to turn a drawn DC
# colour into the stored DC coefficient (the workloads specify colours).
_Y00 = 0.28209479177387814


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # [3,3] float32, world -> camera, row-major
    t: np.ndarray          # [3]   float32
    near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def as_array(self) -> np.ndarray:
        """Packed float32 record: fx fy cx cy R[9] t[3] near bg[3] (20 floats)."""
        return np.concatenate([
            np.array([self.fx, self.fy, self.cx, self.cy], np.float32),
            self.R.astype(np.float32).reshape(9),
            self.t.astype(np.float32).reshape(3),
            np.array([self.near], np.float32),
            np.array(self.bg, np.float32),
        ]).astype(np.float32)


CAMERA_FLOATS = 20


@dataclasses.dataclass
class Scene:
    means: np.ndarray           # [N,3]
    log_scales: np.ndarray      # [N,3]
    quats: np.ndarray           # [N,4] (w,x,y,z)
    opacity_logits: np.ndarray  # [N]
    sh: np.ndarray              # [N,K,3], K=(deg+1)^2
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                     self.opacity_logits.copy(), self.sh.copy(), self.sh_degree)

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cameras: List[Camera]
    target_rgb: Optional[List[np.ndarray]]   # per view [3,H,W] or None
    target_depth: Optional[List[np.ndarray]]  # per view [H,W] or None
    lambda_depth: float
    # Scene whose rendering is the target (None when the target is drawn).
    target_scene: Optional[Scene] = None
    # Ground-truth poses (config 3) before the pose perturbation.
    gt_cameras: Optional[List[Camera]] = None
    pose_perturbation: Optional[np.ndarray] = None   # [V,6] (rho, phi)
    notes: str = ""


# ----------------------------------------------------------------------------
# small helpers (input generation only)
# ----------------------------------------------------------------------------

def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _look_camera(position, forward, width, height, fx, fy, roll=0.0,
                 up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at ``position`` looking along ``forward`` (+y image axis down)."""
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    upv = np.asarray(up, np.float64)
    right = np.cross(f, upv)
    if np.linalg.norm(right) < 1e-6:
        right = np.cross(f, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    if roll != 0.0:
        cr, sr = math.cos(roll), math.sin(roll)
        right, down = cr * right + sr * down, -sr * right + cr * down
    R_cw = np.stack([right, down, f], axis=1)     # camera axes in world
    R = R_cw.T
    t = -R @ np.asarray(position, np.float64)
    return Camera(width, height, float(fx), float(fy), width / 2.0, height / 2.0,
                  _f32(R), _f32(t))


def _yaw_pitch_forward(yaw, pitch):
    return np.array([math.cos(yaw) * math.cos(pitch),
                     math.sin(yaw) * math.cos(pitch),
                     math.sin(pitch)])


def _sh_coeffs(rng, n, degree, dc_colour):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    sh[:, 0, :] = (dc_colour - 0.5) / _Y00
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, k - 1, 3))
    return sh


# ----------------------------------------------------------------------------
# room geometry: rectangles (origin, edge u, edge v) to scatter points on
# ----------------------------------------------------------------------------

def _room_faces(x0, y0, size=(6.0, 5.0, 3.0)):
    sx, sy, sz = size
    o = np.array([x0, y0, 0.0])
    ex, ey, ez = np.array([sx, 0, 0.]), np.array([0, sy, 0.]), np.array([0, 0, sz])
    return [
        (o, ex, ey),               # floor
        (o + ez, ex, ey),          # ceiling
        (o, ex, ez),               # wall y=y0
        (o + ey, ex, ez),          # wall y=y0+sy
        (o, ey, ez),               # wall x=x0
        (o + ex, ey, ez),          # wall x=x0+sx
    ]


def _box_faces(rng, x0, y0, n_boxes, size=(6.0, 5.0, 3.0), margin=0.5):
    faces = []
    sx, sy, _ = size
    for _ in range(n_boxes):
        w, d, h = rng.uniform(0.2, 1.2, size=3)
        cx = rng.uniform(x0 + margin, x0 + sx - margin)
        cy = rng.uniform(y0 + margin, y0 + sy - margin)
        yaw = rng.uniform(0.0, 2 * math.pi)
        a = np.array([math.cos(yaw), math.sin(yaw), 0.0])
        b = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
        z = np.array([0.0, 0.0, 1.0])
        c0 = np.array([cx, cy, 0.0]) - 0.5 * w * a - 0.5 * d * b
        ea, eb, ez = w * a, d * b, h * z
        faces += [
            (c0 + ez, ea, eb),     # top
            (c0, ea, ez),          # side
            (c0 + eb, ea, ez),     # side
            (c0, eb, ez),          # side
            (c0 + ea, eb, ez),     # side
        ]
    return faces


def _scatter_on_faces(rng, faces, n, noise, holes=()):
    """Uniform points on rectangles (count proportional to area) + noise.

    ``holes`` lists axis-aligned boxes (lo, hi) whose points are rejected
    (door openings); rejected points are redrawn from the same face.
    """
    areas = np.array([np.linalg.norm(np.cross(u, v)) for (_, u, v) in faces])
    counts = np.floor(n * areas / areas.sum()).astype(np.int64)
    rem = n - counts.sum()
    order = np.argsort(-(n * areas / areas.sum() - counts), kind="stable")
    counts[order[:rem]] += 1
    pts = []
    for (o, u, v), c in zip(faces, counts):
        got = np.zeros((0, 3))
        while got.shape[0] < c:
            need = c - got.shape[0]
            ab = rng.uniform(0.0, 1.0, size=(need, 2))
            p = o + ab[:, :1] * u + ab[:, 1:] * v
            keep = np.ones(need, bool)
            for lo, hi in holes:
                inside = np.all((p >= np.asarray(lo)) & (p <= np.asarray(hi)), axis=1)
                keep &= ~inside
            got = np.concatenate([got, p[keep]], axis=0)
        pts.append(got[:c])
    pts = np.concatenate(pts, axis=0)
    pts += rng.normal(0.0, noise, size=pts.shape)
    return pts


def _room_gaussians(rng, n, faces, log_scale_mu, log_scale_sigma, degree,
                    holes=(), low_opacity_fraction=0.0):
    means = _scatter_on_faces(rng, faces, n, 0.01, holes)
    perm = rng.permutation(n)               # map order is not spatial order
    means = means[perm]
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = _random_quats(rng, n)
    logits = rng.standard_normal(n)
    if low_opacity_fraction > 0.0:
        sel = rng.uniform(size=n) < low_opacity_fraction
        o = rng.uniform(0.001, 0.05, size=int(sel.sum()))
        logits[sel] = np.log(o / (1.0 - o))
    dc = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _sh_coeffs(rng, n, degree, dc)
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits),
                 _f32(sh), degree)


def _perturbed(rng, scene: Scene) -> Scene:
    """Target-scene perturbation: means, log-scales, DC and opacity logits."""
    s = scene.copy()
    n = s.n
    s.means = _f32(s.means + rng.normal(0.0, 0.005, size=(n, 3)))
    s.log_scales = _f32(s.log_scales + rng.normal(0.0, 0.05, size=(n, 3)))
    sh = s.sh.astype(np.float64)
    sh[:, 0, :] += rng.normal(0.0, 0.05, size=(n, 3)) / _Y00
    s.sh = _f32(sh)
    s.opacity_logits = _f32(s.opacity_logits + rng.normal(0.0, 0.2, size=n))
    return s


def _inside_room_camera(rng, width, height, f, x0=0.0, y0=0.0):
    pos = np.array([x0 + rng.uniform(1, 5), y0 + rng.uniform(1, 4), rng.uniform(1.2, 1.8)])
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = rng.normal(0.0, 0.15)
    roll = rng.normal(0.0, 0.05)
    return _look_camera(pos, _yaw_pitch_forward(yaw, pitch), width, height, f, f, roll)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def slab_128x96(seed: int = 1001, n: int = 2000) -> Workload:
    """128x96, fx=fy=100, identity pose, N Gaussians in x,y in [-1,1], z in [2,4]."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 4, n)], 1)
    log_scales = rng.normal(-3.0, 0.3, size=(n, 3))
    quats = _random_quats(rng, n)
    logits = rng.standard_normal(n)
    colour = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _sh_coeffs(rng, n, 0, colour)
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 0)
    cam = Camera(128, 96, 100.0, 100.0, 64.0, 48.0, _f32(np.eye(3)), _f32(np.zeros(3)))
    target = _f32(rng.uniform(0.0, 1.0, size=(3, 96, 128)))
    return Workload("slab_128x96_2k_sh0", scene, [cam], [target], None, 0.0,
                    notes="L1 RGB against a uniform random target")


def room_1200x680(seed: int = 1002, n: int = 300_000, width: int = 1200, height: int = 680,
            f: float = 600.0) -> Workload:
    rng = np.random.default_rng(seed)
    faces = _room_faces(0.0, 0.0) + _box_faces(rng, 0.0, 0.0, 20)
    scene = _room_gaussians(rng, n, faces, -4.5, 0.4, 3)
    cam = _inside_room_camera(rng, width, height, f)
    target_scene = _perturbed(rng, scene)
    return Workload("room_1200x680_300k_sh3", scene, [cam], None, None, 0.1,
                    target_scene=target_scene,
                    notes="L1 RGB + 0.1 L1 depth against a render of perturbed params")


def _so3(phi):
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(np.asarray(phi, np.float64)).as_matrix()


def perturb_camera(cam: Camera, xi) -> Camera:
    """Left perturbation of the world->camera pose by xi=(rho, phi):
    R' = Exp(phi) R, t' = Exp(phi) t + rho."""
    Rp = _so3(xi[3:6])
    R = Rp @ cam.R.astype(np.float64)
    t = Rp @ cam.t.astype(np.float64) + np.asarray(xi[0:3], np.float64)
    return dataclasses.replace(cam, R=_f32(R), t=_f32(t))


def room_640x480_pose(seed: int = 1003, n: int = 150_000) -> Workload:
    rng = np.random.default_rng(seed)
    faces = _room_faces(0.0, 0.0) + _box_faces(rng, 0.0, 0.0, 20)
    scene = _room_gaussians(rng, n, faces, -4.5, 0.4, 3)
    gt = _inside_room_camera(rng, 640, 480, 525.0)
    xi = np.concatenate([rng.normal(0.0, 0.02, 3), rng.normal(0.0, 0.01, 3)])
    cam = perturb_camera(gt, xi)
    return Workload("room_640x480_150k_sh3_pose", scene, [cam], None, None, 0.1,
                    target_scene=scene, gt_cameras=[gt], pose_perturbation=xi[None, :],
                    notes="target rendered at the ground-truth pose")


def _closeup_camera(rng, width, height, f, x0, y0, size=(6.0, 5.0, 3.0)):
    sx, sy, _ = size
    wall = int(rng.integers(0, 4))
    dist = rng.uniform(0.4, 0.8)
    z = rng.uniform(0.8, 2.0)
    if wall == 0:
        pos, fwd = (x0 + rng.uniform(1, sx - 1), y0 + dist, z), (0, -1, 0)
    elif wall == 1:
        pos, fwd = (x0 + rng.uniform(1, sx - 1), y0 + sy - dist, z), (0, 1, 0)
    elif wall == 2:
        pos, fwd = (x0 + dist, y0 + rng.uniform(1, sy - 1), z), (-1, 0, 0)
    else:
        pos, fwd = (x0 + sx - dist, y0 + rng.uniform(1, sy - 1), z), (1, 0, 0)
    fwd = np.asarray(fwd, np.float64) + rng.normal(0.0, 0.05, 3)
    return _look_camera(np.asarray(pos), fwd, width, height, f, f, rng.normal(0.0, 0.03))


def _overview_camera(rng, width, height, f, x0, y0, size=(6.0, 5.0, 3.0)):
    sx, sy, sz = size
    corner = int(rng.integers(0, 4))
    cxs = [x0 + 0.3, x0 + sx - 0.3]
    cys = [y0 + 0.3, y0 + sy - 0.3]
    px, py = cxs[corner & 1], cys[corner >> 1]
    pos = np.array([px, py, sz - 0.4])
    centre = np.array([x0 + sx / 2, y0 + sy / 2, 0.6])
    fwd = centre - pos + rng.normal(0.0, 0.1, 3)
    return _look_camera(pos, fwd, width, height, f, f, rng.normal(0.0, 0.03))


_RESOLUTIONS = [(640, 480), (1200, 680), (320, 240)]


def keyframes8_mixed(seed: int = 1004, n: int = 500_000, n_views: int = 8) -> Workload:
    """8 keyframes, mixed resolution, alternating close-up / overview poses."""
    rng = np.random.default_rng(seed)
    faces = _room_faces(0.0, 0.0) + _box_faces(rng, 0.0, 0.0, 20)
    scene = _room_gaussians(rng, n, faces, -4.5, 0.4, 3)
    cams = []
    for v in range(n_views):
        w, h = _RESOLUTIONS[int(rng.integers(0, 3))]
        if v % 2 == 0:
            cams.append(_closeup_camera(rng, w, h, w / 2.0, 0.0, 0.0))
        else:
            cams.append(_overview_camera(rng, w, h, w / 2.0, 0.0, 0.0))
    target_scene = _perturbed(rng, scene)
    return Workload("keyframes8_mixed_500k_sh3", scene, cams, None, None, 0.1,
                    target_scene=target_scene,
                    notes="batched keyframes; targets are renders of perturbed params")


def keyframes16_1200x680(seed: int = 1005, n: int = 2_000_000, n_views: int = 16) -> Workload:
    """Four 6x5x3 rooms in a 2x2 layout with 1 m doorways, 16 views."""
    rng = np.random.default_rng(seed)
    faces, holes = [], []
    for ry in range(2):
        for rx in range(2):
            faces += _room_faces(6.0 * rx, 5.0 * ry) + _box_faces(rng, 6.0 * rx, 5.0 * ry, 20)
    # doorways through the shared walls x=6 and y=5 (1 m wide, 2.1 m high)
    for yc in (2.5, 7.5):
        holes.append(((5.9, yc - 0.5, -0.1), (6.1, yc + 0.5, 2.1)))
    for xc in (3.0, 9.0):
        holes.append(((xc - 0.5, 4.9, -0.1), (xc + 0.5, 5.1, 2.1)))
    scene = _room_gaussians(rng, n, faces, -5.0, 0.5, 3, holes=holes,
                            low_opacity_fraction=0.3)
    cams = []
    for v in range(n_views):
        room = v // (n_views // 4) if n_views >= 4 else 0
        x0, y0 = 6.0 * (room & 1), 5.0 * (room >> 1)
        cams.append(_inside_room_camera(rng, 1200, 680, 600.0, x0, y0))
    target_scene = _perturbed(rng, scene)
    return Workload("keyframes16_1200x680_2M_sh3", scene, cams, None, None, 0.1,
                    target_scene=target_scene,
                    notes="large scene; forward + backward + Adam per iteration")


def keyframe_pool_640x480(seed: int = 1006, n: int = 150_000, n_keyframes: int = 6) -> Workload:
    """A pool of keyframes of one 640x480 camera inside the room (the
    keyframes a scheduled batch draws from); targets are renders of
    perturbed parameters."""
    rng = np.random.default_rng(seed)
    faces = _room_faces(0.0, 0.0) + _box_faces(rng, 0.0, 0.0, 20)
    scene = _room_gaussians(rng, n, faces, -4.5, 0.4, 3)
    cams = [_inside_room_camera(rng, 640, 480, 525.0) for _ in range(n_keyframes)]
    target_scene = _perturbed(rng, scene)
    return Workload("keyframe_pool_640x480_150k_sh3", scene, cams, None, None, 0.1,
                    target_scene=target_scene,
                    notes="keyframe pool for scheduled batches")


def tiny_scene(seed: int, n: int = 8, width: int = 32, height: int = 24,
               degree: int = 0, f: float = 30.0) -> Workload:
    """Small scene for finite-difference checks: Gaussians in front of an
    identity camera with moderate scales so each covers several pixels."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.45, 0.45, n),
                      rng.uniform(2.0, 3.0, n)], 1)
    log_scales = rng.normal(-2.3, 0.25, size=(n, 3))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.0, 0.8, size=n)
    colour = rng.uniform(0.1, 0.9, size=(n, 3))
    sh = _sh_coeffs(rng, n, degree, colour)
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), degree)
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0, _f32(np.eye(3)), _f32(np.zeros(3)))
    return Workload(f"tiny_{seed}", scene, [cam], None, None, 0.0)


def crowded_scene(seed: int, n: int = 6000, width: int = 64, height: int = 48,
                  degree: int = 1, f: float = 60.0) -> Workload:
    """Many faint, small Gaussians stacked over a few tiles: per-tile lists of
    thousands of pairs (long-list sorting, long compositing chains)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(2.0, 3.0, n)
    # screen positions around pixel (21, 19), spread +-2.5 px
    u = 21.0 + rng.uniform(-2.5, 2.5, n)
    v = 19.0 + rng.uniform(-2.5, 2.5, n)
    means = np.stack([(u - width / 2.0) * z / f, (v - height / 2.0) * z / f, z], 1)
    log_scales = rng.normal(-4.2, 0.15, size=(n, 3))
    quats = _random_quats(rng, n)
    logits = rng.normal(-3.2, 0.2, size=n)
    colour = rng.uniform(0.1, 0.9, size=(n, 3))
    sh = _sh_coeffs(rng, n, degree, colour)
    scene = Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), degree)
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0, _f32(np.eye(3)), _f32(np.zeros(3)))
    return Workload(f"crowded_{seed}", scene, [cam], None, None, 0.0)


def random_pose(rng, scale_rot=0.2, scale_trans=0.3):
    """A random world->camera rigid transform near identity (for invariance tests)."""
    R = _so3(rng.normal(0.0, scale_rot, 3))
    t = rng.normal(0.0, scale_trans, 3)
    return R, t


def linear_loss_weights(seed: int, cameras: List[Camera]):
    """Fixed random upstream gradients dL/dC [3,H,W] and dL/dD [H,W] per view
    (a linear loss, free of L1 kinks, for gradient parity)."""
    rng = np.random.default_rng(seed)
    gc, gd = [], []
    for cam in cameras:
        npx = cam.width * cam.height
        gc.append(_f32(rng.standard_normal((3, cam.height, cam.width)) / npx))
        gd.append(_f32(rng.standard_normal((cam.height, cam.width)) / npx))
    return gc, gd


def random_keys(seed: int, n: int, tile_bits: int, tie_fraction: float = 0.05):
    """Synthetic (tile, depth) sort keys with deliberate depth ties, as uint64,
    and values 0..n-1 (uint32).  Depths are positive float32 bit patterns."""
    rng = np.random.default_rng(seed)
    tiles = rng.integers(0, 1 << tile_bits, size=n, dtype=np.uint64)
    depth = rng.uniform(0.2, 50.0, size=n).astype(np.float32)
    k = int(n * tie_fraction)
    if k > 0 and n > 1:
        src = rng.integers(0, n, size=k)
        dst = rng.integers(0, n, size=k)
        depth[dst] = depth[src]
        tiles[dst] = tiles[src]
    bits = depth.view(np.uint32).astype(np.uint64)
    keys = (tiles << np.uint64(32)) | bits
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


WORKLOADS = {1: slab_128x96, 2: room_1200x680, 3: room_640x480_pose, 4: keyframes8_mixed, 5: keyframes16_1200x680}
