"""Seeded synthetic surfel scenes, cameras and poses.

Conventions shared by every consumer of these arrays:

* Surfels are a structure-of-arrays ``float32[15, N]`` in row order
  mu.xyz, t_u.xyz, t_v.xyz, s_u, s_v, opacity, r, g, b.  Scales and opacity are
  post-activation values; colour is a plain RGB triple (the paper drops
  spherical harmonics, Sec. "Camera Pose Optimization").
* A pose is a ``float32[3, 4]`` matrix [R | t] mapping world points into the
  camera frame (x right, y down, z forward).
* A camera is (width, height, fx, fy, cx, cy); pixel (x, y) is sampled at the
  integer image coordinates x, y.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.  Rotations
used to build or perturb poses come from ``scipy.spatial.transform.Rotation``
so that this module carries no Lie-group code of its own.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

PARAM_ROWS = 15


@dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy)


@dataclass
class SurfelSet:
    """Surfels in the [15, N] float32 layout plus the pose and camera to view them."""

    params: np.ndarray
    camera: Camera
    pose: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.params.shape[1])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pack(mu, tu, tv, su, sv, o, rgb) -> np.ndarray:
    n = mu.shape[0]
    p = np.empty((PARAM_ROWS, n), dtype=np.float32)
    p[0:3] = mu.T
    p[3:6] = tu.T
    p[6:9] = tv.T
    p[9] = su
    p[10] = sv
    p[11] = o
    p[12:15] = rgb.T
    return p


def _identity_pose() -> np.ndarray:
    return np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).astype(np.float32)


def random_surfels(n: int = 2000, seed: int = 0, camera: Camera | None = None) -> SurfelSet:
    """Random surfels in front of a small pinhole camera (the 64x48 single-frame workload).

    Centres uniform in [-1,1]x[-1,1]x[2,4]; t_u uniform on the sphere; t_v the
    normalised component of a Gaussian vector orthogonal to t_u; scales
    log-uniform in [0.01, 0.1]; opacity sigmoid(N(0,1)); RGB uniform in [0,1].
    """
    g = _rng(seed)
    cam = camera or Camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    mu = np.stack([g.uniform(-1, 1, n), g.uniform(-1, 1, n), g.uniform(2, 4, n)], axis=1)
    tu = g.normal(size=(n, 3))
    tu /= np.linalg.norm(tu, axis=1, keepdims=True)
    gv = g.normal(size=(n, 3))
    tv = gv - np.sum(gv * tu, axis=1, keepdims=True) * tu
    tv /= np.linalg.norm(tv, axis=1, keepdims=True)
    su = np.exp(g.uniform(np.log(0.01), np.log(0.1), n))
    sv = np.exp(g.uniform(np.log(0.01), np.log(0.1), n))
    o = 1.0 / (1.0 + np.exp(-g.normal(size=n)))
    rgb = g.uniform(0, 1, (n, 3))
    return SurfelSet(_pack(mu, tu, tv, su, sv, o, rgb), cam, _identity_pose(),
                     {"workload": "random", "seed": seed})


def single_surfel(scale: float = 0.1, opacity: float = 0.8, rgb=(0.2, 0.4, 0.6),
                  depth: float = 2.0) -> SurfelSet:
    """One fronto-parallel surfel on the optical axis of a 64x48, f=60 camera."""
    cam = Camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    mu = np.array([[0.0, 0.0, depth]])
    tu = np.array([[1.0, 0.0, 0.0]])
    tv = np.array([[0.0, 1.0, 0.0]])
    p = _pack(mu, tu, tv, np.array([scale]), np.array([scale]), np.array([opacity]),
              np.array([rgb]))
    return SurfelSet(p, cam, _identity_pose(), {"workload": "single"})


def stacked_surfels(count: int = 20, opacity: float = 0.5, z0: float = 2.0, dz: float = 0.1,
                    width_px: float = 3.0) -> SurfelSet:
    """``count`` fronto-parallel surfels on the optical axis at z0 + k*dz.

    Each is ``width_px`` pixels wide (one sigma) at its own depth and has colour
    (k, 0, 0)/count so that composited members can be told apart.
    """
    cam = Camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    k = np.arange(count, dtype=np.float64)
    z = z0 + dz * k
    mu = np.stack([np.zeros(count), np.zeros(count), z], axis=1)
    tu = np.tile([1.0, 0.0, 0.0], (count, 1))
    tv = np.tile([0.0, 1.0, 0.0], (count, 1))
    s = width_px * z / cam.fx
    rgb = np.stack([k / count, np.zeros(count), np.zeros(count)], axis=1)
    p = _pack(mu, tu, tv, s, s, np.full(count, opacity), rgb)
    return SurfelSet(p, cam, _identity_pose(), {"workload": "stacked"})


def look_at_pose(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera pose [R|t] for a camera at ``eye`` looking at ``target``.

    Camera axes: x right, y down, z forward (towards ``target``).
    """
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    r_wc = np.stack([right, down, fwd], axis=1)
    r_cw = r_wc.T
    t = -r_cw @ eye
    return np.concatenate([r_cw, t[:, None]], axis=1).astype(np.float32)


def planar_carpet(obliquity_deg: float, azimuth_deg: float = 0.0, distance: float = 2.0,
                  spacing: float = 0.02, size: float = 1.0, scale: float = 0.02,
                  camera: Camera | None = None, seed: int = 0) -> SurfelSet:
    """A square grid of coplanar surfels sharing one tangent frame, viewed obliquely.

    The carpet lies in the world plane z = 0 with normal -z (pointing away
    from a viewer above it).  The camera sits ``distance`` metres from the carpet
    centre, its view ray making ``obliquity_deg`` with the plane normal.
    ``info`` holds the plane (normal n, offset h with n.X = h for world X).
    """
    cam = camera or Camera(320, 240, 300.0, 300.0, 160.0, 120.0)
    g = _rng(seed)
    m = int(round(size / spacing)) + 1
    xs = (np.arange(m) - (m - 1) / 2) * spacing
    gx, gy = np.meshgrid(xs, xs, indexing="ij")
    n = m * m
    mu = np.stack([gx.ravel(), gy.ravel(), np.zeros(n)], axis=1)
    theta = g.uniform(0, 2 * np.pi)
    tu1 = np.array([np.cos(theta), np.sin(theta), 0.0])
    normal = np.array([0.0, 0.0, -1.0])
    tv1 = np.cross(normal, tu1)
    tu = np.tile(tu1, (n, 1))
    tv = np.tile(tv1, (n, 1))
    rgb = g.uniform(0, 1, (n, 3))
    p = _pack(mu, tu, tv, np.full(n, scale), np.full(n, scale), np.full(n, 0.7), rgb)
    ob = np.deg2rad(obliquity_deg)
    az = np.deg2rad(azimuth_deg)
    eye = distance * np.array([np.sin(ob) * np.cos(az), np.sin(ob) * np.sin(az), np.cos(ob)])
    pose = look_at_pose(eye, np.zeros(3), up=(0.0, 1.0, 0.0) if obliquity_deg < 1e-6 else (0.0, 0.0, 1.0))
    return SurfelSet(p, cam, pose, {"workload": "carpet", "plane_normal": normal, "plane_offset": 0.0})


def tiny_scene(seed: int, n: int = 4, width: int = 24, height: int = 20,
               focal: float = 30.0) -> SurfelSet:
    """A handful of large, random surfels filling a tiny image (finite-difference scenes)."""
    g = _rng(seed)
    cam = Camera(width, height, focal, focal, width / 2.0, height / 2.0)
    z = g.uniform(1.5, 3.0, n)
    mu = np.stack([g.uniform(-0.25, 0.25, n) * z, g.uniform(-0.25, 0.25, n) * z, z], axis=1)
    tu = g.normal(size=(n, 3))
    tu /= np.linalg.norm(tu, axis=1, keepdims=True)
    gv = g.normal(size=(n, 3))
    tv = gv - np.sum(gv * tu, axis=1, keepdims=True) * tu
    tv /= np.linalg.norm(tv, axis=1, keepdims=True)
    su = np.exp(g.uniform(np.log(0.08), np.log(0.3), n))
    sv = np.exp(g.uniform(np.log(0.08), np.log(0.3), n))
    o = g.uniform(0.3, 0.9, n)
    rgb = g.uniform(0, 1, (n, 3))
    # a small rotation and translation so the pose is not the identity
    rot = Rotation.from_rotvec(g.normal(size=3) * 0.05).as_matrix()
    t = g.normal(size=3) * 0.05
    pose = np.concatenate([rot, t[:, None]], axis=1).astype(np.float32)
    # move the surfels so that they sit where the identity camera would see them
    mu_w = (rot.T @ (mu.T - t[:, None])).T
    tu_w = (rot.T @ tu.T).T
    tv_w = (rot.T @ tv.T).T
    return SurfelSet(_pack(mu_w, tu_w, tv_w, su, sv, o, rgb), cam, pose,
                     {"workload": "tiny", "seed": seed})


# ----------------------------------------------------------------------------------
# Synthetic rooms shaped like indoor RGB-D sequences
# ----------------------------------------------------------------------------------

@dataclass
class Room:
    params: np.ndarray            # float32 [15, N]
    boxes: np.ndarray             # float64 [B, 6]: x0, y0, x1, y1, height (z0 = 0), unused
    extent: tuple                 # room size (X, Y, Z)
    seed: int

    @property
    def n(self) -> int:
        return int(self.params.shape[1])


def _faces(extent, boxes):
    """Faces as (origin, edge1, edge2, normal-away-from-free-space, owner) tuples."""
    X, Y, Z = extent
    f = []
    ex, ey, ez = np.eye(3)
    # room interior: normals point out of the room (away from the free space inside)
    f.append((np.zeros(3), X * ex, Y * ey, -ez, -1))                 # floor
    f.append((np.array([0, 0, Z]), X * ex, Y * ey, ez, -1))          # ceiling
    f.append((np.zeros(3), X * ex, Z * ez, -ey, -1))                 # wall y = 0
    f.append((np.array([0, Y, 0]), X * ex, Z * ez, ey, -1))          # wall y = Y
    f.append((np.zeros(3), Y * ey, Z * ez, -ex, -1))                 # wall x = 0
    f.append((np.array([X, 0, 0]), Y * ey, Z * ez, ex, -1))          # wall x = X
    for b, (x0, y0, x1, y1, h, _) in enumerate(boxes):
        dx, dy = x1 - x0, y1 - y0
        # box surfaces: normals point into the box (away from the free space outside)
        f.append((np.array([x0, y0, h]), dx * ex, dy * ey, -ez, b))   # top
        f.append((np.array([x0, y0, 0]), dx * ex, h * ez, ey, b))     # side y = y0
        f.append((np.array([x0, y1, 0]), dx * ex, h * ez, -ey, b))    # side y = y1
        f.append((np.array([x0, y0, 0]), dy * ey, h * ez, ex, b))     # side x = x0
        f.append((np.array([x1, y0, 0]), dy * ey, h * ez, -ex, b))    # side x = x1
    return f


def _inside_any(p, boxes, skip):
    """Boolean mask: points strictly inside (or under) a box other than their own."""
    out = np.zeros(p.shape[0], dtype=bool)
    eps = 1e-9
    for b, (x0, y0, x1, y1, h, _) in enumerate(boxes):
        m = ((p[:, 0] > x0 + eps) & (p[:, 0] < x1 - eps) & (p[:, 1] > y0 + eps)
             & (p[:, 1] < y1 - eps) & (p[:, 2] < h - eps))
        out |= m & (skip != b)
    return out


def make_room(n: int, seed: int = 0, extent=(6.0, 5.0, 3.0), n_boxes: int = 20,
              scale_range=(0.005, 0.03), opacity: float = 0.95) -> Room:
    """A box-shaped room with ``n_boxes`` axis-aligned boxes on its floor, covered by ``n`` surfels.

    Points are drawn area-weighted over every face; points that fall inside or
    under another box are redrawn until exactly ``n`` remain.  Each surfel's
    normal t_u x t_v points away from the free space, t_u is uniform in the face
    plane, scales are log-uniform in ``scale_range`` and colour is a smooth
    sum of three sinusoids per channel.
    """
    g = _rng(seed)
    X, Y, Z = extent
    boxes = []
    for _ in range(n_boxes):
        sx, sy = g.uniform(0.2, 1.0, 2)
        h = g.uniform(0.2, 1.5)
        x0 = g.uniform(0.3, X - 0.3 - sx)
        y0 = g.uniform(0.3, Y - 0.3 - sy)
        boxes.append((x0, y0, x0 + sx, y0 + sy, h, 0.0))
    boxes = np.array(boxes, dtype=np.float64).reshape(-1, 6)
    faces = _faces(extent, boxes)
    areas = np.array([np.linalg.norm(e1) * np.linalg.norm(e2) for _, e1, e2, _, _ in faces])
    prob = areas / areas.sum()

    pts, nrm, e1s, e2s = [], [], [], []
    have = 0
    while have < n:
        m = int((n - have) * 1.3) + 64
        fi = g.choice(len(faces), size=m, p=prob)
        r = g.uniform(0, 1, (m, 2))
        org = np.stack([faces[i][0] for i in fi])
        e1 = np.stack([faces[i][1] for i in fi])
        e2 = np.stack([faces[i][2] for i in fi])
        nn = np.stack([faces[i][3] for i in fi])
        own = np.array([faces[i][4] for i in fi])
        p = org + r[:, :1] * e1 + r[:, 1:2] * e2
        keep = ~_inside_any(p, boxes, own)
        take = min(int(keep.sum()), n - have)
        idx = np.nonzero(keep)[0][:take]
        pts.append(p[idx]); nrm.append(nn[idx]); e1s.append(e1[idx]); e2s.append(e2[idx])
        have += take
    p = np.concatenate(pts)
    nn = np.concatenate(nrm)
    e1 = np.concatenate(e1s)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nn, e1)
    ang = g.uniform(0, 2 * np.pi, n)
    tu = np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2
    tv = np.cross(nn, tu)
    su = np.exp(g.uniform(np.log(scale_range[0]), np.log(scale_range[1]), n))
    sv = np.exp(g.uniform(np.log(scale_range[0]), np.log(scale_range[1]), n))
    o = np.full(n, opacity)
    rgb = np.empty((n, 3))
    for c in range(3):
        acc = np.full(n, 0.5)
        for _ in range(3):
            d = g.normal(size=3)
            d /= np.linalg.norm(d)
            f = d * g.uniform(0.2, 1.0)
            ph = g.uniform(0, 2 * np.pi)
            acc += np.sin(2 * np.pi * (p @ f) + ph) / 6.0
        rgb[:, c] = np.clip(acc, 0.0, 1.0)
    params = _pack(p, tu, tv, su, sv, o, rgb)
    return Room(params, boxes, tuple(extent), seed)


def _dist_to_box(c, box):
    x0, y0, x1, y1, h, _ = box
    lo = np.array([x0, y0, 0.0])
    hi = np.array([x1, y1, h])
    d = np.maximum(np.maximum(lo - c, 0.0), c - hi)
    return float(np.linalg.norm(d))


def room_camera(room: Room, seed: int, min_clearance: float = 0.5) -> np.ndarray:
    """A ground-truth world->camera pose inside ``room``.

    Camera centre uniform in [1.5,4.5]x[1.5,3.5]x[1.2,1.8] (scaled to the room
    extent) and at least ``min_clearance`` from every box; yaw uniform, pitch
    uniform in [-15, 15] degrees, no roll.
    """
    g = _rng(seed)
    X, Y, _ = room.extent
    for _ in range(10000):
        c = np.array([g.uniform(1.5, X - 1.5), g.uniform(1.5, Y - 1.5), g.uniform(1.2, 1.8)])
        if all(_dist_to_box(c, b) >= min_clearance for b in room.boxes):
            break
    else:  # pragma: no cover - rooms with 20 boxes always have free space
        raise RuntimeError("no free camera position")
    yaw = g.uniform(0, 2 * np.pi)
    pitch = np.deg2rad(g.uniform(-15, 15))
    fwd = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
    return look_at_pose(c, c + fwd)


def perturb_pose(pose: np.ndarray, trans_m: float, rot_deg: float, seed: int) -> np.ndarray:
    """Move the camera centre by ``trans_m`` and rotate the camera by ``rot_deg``.

    Directions are uniform; the rotation is applied on the camera side
    (R' = R_delta R), so the camera-centre distance and the rotation angle
    between the two poses are exactly the requested magnitudes.
    """
    g = _rng(seed)
    pose = np.asarray(pose, dtype=np.float64)
    r, t = pose[:, :3], pose[:, 3]
    c = -r.T @ t
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    ax = g.normal(size=3)
    ax /= np.linalg.norm(ax)
    r_new = Rotation.from_rotvec(ax * np.deg2rad(rot_deg)).as_matrix() @ r
    c_new = c + trans_m * d
    return np.concatenate([r_new, (-r_new @ c_new)[:, None]], axis=1).astype(np.float32)


def pose_error(est: np.ndarray, gt: np.ndarray):
    """(camera-centre distance in metres, rotation angle in degrees) between two poses."""
    est = np.asarray(est, dtype=np.float64)
    gt = np.asarray(gt, dtype=np.float64)
    ce = -est[:, :3].T @ est[:, 3]
    cg = -gt[:, :3].T @ gt[:, 3]
    rel = est[:, :3] @ gt[:, :3].T
    # re-orthonormalise before measuring the angle (poses are stored in float32)
    u, _, vt = np.linalg.svd(rel)
    ang = Rotation.from_matrix(u @ vt).magnitude()
    return float(np.linalg.norm(ce - cg)), float(np.rad2deg(ang))
