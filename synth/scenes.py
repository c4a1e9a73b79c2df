"""Scene synthesis for the four workload shapes used by tests and benchmarks.

All generators are seeded (NumPy ``Generator(PCG64)``) and return FP32 SoA
clouds of shape ``(3, N)``.  Every pair carries the rigid transform that maps
the *target* cloud into the *source* frame (``src ~= R_true @ tgt + t_true``),
which is what registering the target against a model of the source recovers
(the problem statement of Sec. 3, Eq. 1: the model is built from the first
cloud, the second cloud is moved onto it).

Workload shapes (the paper's datasets are not available; these stand in):

* ``small_pair``   -- planes and spheres in the unit cube, 10k points per
  cloud, stands in for the Stanford Bunny experiment of Sec. 5.
* ``lidar_pair``   -- a 64-ring x 1875-azimuth spinning scan of a street-like
  scene, stands in for the Velodyne sweeps of Sec. 6.
* ``depth_pair``   -- a 640x480 depth camera in a furnished room, stands in for
  the Lounge (Kinect) sequence of Sec. 6.
* ``uneven_batch`` -- 256 ``small_pair``-style pairs with log-uniform sizes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# small helpers (pose synthesis only)
# --------------------------------------------------------------------------

def rotation_from_axis_angle(axis, angle_rad: float) -> np.ndarray:
    """Rotation matrix from a unit axis and an angle (Rodrigues' formula)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle_rad) * k + (1.0 - math.cos(angle_rad)) * (k @ k)


def rotation_angle_deg(R_est: np.ndarray, R_true: np.ndarray) -> float:
    """Geodesic angle between two rotations, in degrees."""
    c = (np.trace(np.asarray(R_est) @ np.asarray(R_true).T) - 1.0) * 0.5
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def _unit_sphere(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    w = np.asarray(weights, dtype=np.float64)
    q = w / w.sum() * total
    base = np.floor(q).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return base


def as_soa(points_n3: np.ndarray) -> np.ndarray:
    """(N,3) -> contiguous FP32 (3,N)."""
    return np.ascontiguousarray(np.asarray(points_n3, dtype=np.float32).T)


@dataclass
class PairSample:
    src: np.ndarray          # (3, N1) float32, the model cloud Z1
    tgt: np.ndarray          # (3, N2) float32, the cloud Z2 to register
    R_true: np.ndarray       # (3, 3) float64: src ~= R_true @ tgt + t_true
    t_true: np.ndarray       # (3,) float64
    extent: float            # bounding-box diagonal of src
    meta: dict = field(default_factory=dict)


@dataclass
class BatchSample:
    src: np.ndarray          # (3, sum N) float32, CSR by src_offsets
    tgt: np.ndarray          # (3, sum N) float32, CSR by tgt_offsets
    src_offsets: np.ndarray  # (B+1,) int64
    tgt_offsets: np.ndarray  # (B+1,) int64
    levels: np.ndarray       # (B,) int32
    R_true: np.ndarray       # (B, 3, 3)
    t_true: np.ndarray       # (B, 3)
    meta: dict = field(default_factory=dict)


def _extent(p_soa: np.ndarray) -> float:
    lo = p_soa.min(axis=1).astype(np.float64)
    hi = p_soa.max(axis=1).astype(np.float64)
    return float(np.linalg.norm(hi - lo))


# --------------------------------------------------------------------------
# planes + spheres in the unit cube (small / batched / warm-start shapes)
# --------------------------------------------------------------------------

_HALF = 0.5
_PATCH = math.sqrt(3.0)


def _plane_frame(normal):
    n = normal / np.linalg.norm(normal)
    helper = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(n, helper)
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    return u, v


def _cube_scene(rng: np.random.Generator, n_planes=4, n_spheres=2):
    planes = []
    for _ in range(n_planes):
        normal = _unit_sphere(rng, 1)[0]
        anchor = rng.uniform(-0.25, 0.25, size=3)
        u, v = _plane_frame(normal)
        # fraction of the sqrt(3)-side patch that lies inside the cube,
        # estimated once per plane from the scene stream
        st = rng.uniform(-_PATCH / 2, _PATCH / 2, size=(4096, 2))
        pts = anchor + st[:, :1] * u + st[:, 1:] * v
        frac = np.mean(np.all(np.abs(pts) <= _HALF, axis=1))
        planes.append(dict(anchor=anchor, u=u, v=v, area=_PATCH * _PATCH * max(frac, 1e-3)))
    spheres = []
    for _ in range(n_spheres):
        r = rng.uniform(0.1, 0.3)
        c = rng.uniform(-_HALF + r, _HALF - r, size=3)
        spheres.append(dict(center=c, radius=r, area=4.0 * math.pi * r * r))
    return planes, spheres


def _sample_cube_scene(planes, spheres, n, rng):
    areas = np.array([p["area"] for p in planes] + [s["area"] for s in spheres])
    counts = _largest_remainder(areas, n)
    out = []
    for p, c in zip(planes, counts[: len(planes)]):
        got = []
        need = int(c)
        while need > 0:
            st = rng.uniform(-_PATCH / 2, _PATCH / 2, size=(max(2 * need, 64), 2))
            pts = p["anchor"] + st[:, :1] * p["u"] + st[:, 1:] * p["v"]
            pts = pts[np.all(np.abs(pts) <= _HALF, axis=1)][:need]
            got.append(pts)
            need -= len(pts)
        out.append(np.concatenate(got) if got else np.zeros((0, 3)))
    for s, c in zip(spheres, counts[len(planes):]):
        out.append(s["center"] + s["radius"] * _unit_sphere(rng, int(c)))
    return np.concatenate(out, axis=0)


def small_pair(seed: int, n: int = 10_000, max_angle_deg: float = 30.0,
               max_trans: float = 0.1, noise: float = 0.005,
               n_tgt: int | None = None) -> PairSample:
    """Planes + spheres in [-0.5, 0.5]^3; target = independent resample, rigidly moved.

    Streams (SeedSequence(seed).spawn(5)): scene, source sampling, target
    sampling, noise, pose.
    """
    s_scene, s_src, s_tgt, s_noise, s_pose = [
        np.random.Generator(np.random.PCG64(ss)) for ss in np.random.SeedSequence(seed).spawn(5)
    ]
    planes, spheres = _cube_scene(s_scene)
    src = _sample_cube_scene(planes, spheres, n, s_src)
    tgt = _sample_cube_scene(planes, spheres, n if n_tgt is None else n_tgt, s_tgt)
    src = src + s_noise.normal(0.0, noise, size=src.shape)
    tgt = tgt + s_noise.normal(0.0, noise, size=tgt.shape)
    axis = _unit_sphere(s_pose, 1)[0]
    ang = math.radians(s_pose.uniform(0.0, max_angle_deg))
    Rg = rotation_from_axis_angle(axis, ang)
    tg = s_pose.uniform(-max_trans, max_trans, size=3)
    tgt = tgt @ Rg.T + tg
    src32 = as_soa(src)
    return PairSample(src=src32, tgt=as_soa(tgt), R_true=Rg.T.copy(), t_true=-(Rg.T @ tg),
                      extent=_extent(src32),
                      meta=dict(kind="small", seed=seed, n=n, angle_deg=math.degrees(ang)))


# --------------------------------------------------------------------------
# spinning LiDAR in a street-like scene
# --------------------------------------------------------------------------

def _ray_boxes(o, d, boxes):
    """Nearest positive hit of rays (o + t d) with axis-aligned boxes; inf on miss."""
    best = np.full(d.shape[0], np.inf)
    inv = 1.0 / np.where(np.abs(d) < 1e-12, 1e-12, d)
    for lo, hi in boxes:
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
        tmin = np.max(np.minimum(t1, t2), axis=1)
        tmax = np.min(np.maximum(t1, t2), axis=1)
        hit = (tmax >= tmin) & (tmax > 0)
        t = np.where(tmin > 1e-6, tmin, tmax)
        best = np.where(hit & (t < best), t, best)
    return best


def _ray_cylinders(o, d, cyls):
    best = np.full(d.shape[0], np.inf)
    for cx, cy, r, h in cyls:
        ox, oy = o[0] - cx, o[1] - cy
        a = d[:, 0] ** 2 + d[:, 1] ** 2
        b = 2 * (ox * d[:, 0] + oy * d[:, 1])
        c = ox * ox + oy * oy - r * r
        disc = b * b - 4 * a * c
        ok = (disc >= 0) & (a > 1e-12)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t = (-b - sq) / np.where(ok, 2 * a, 1.0)
        z = o[2] + t * d[:, 2]
        side = ok & (t > 1e-6) & (z >= 0) & (z <= h)
        # top cap
        tc = (h - o[2]) / np.where(np.abs(d[:, 2]) < 1e-12, 1e-12, d[:, 2])
        xc = ox + tc * d[:, 0]
        yc = oy + tc * d[:, 1]
        cap = (tc > 1e-6) & (xc * xc + yc * yc <= r * r)
        tt = np.where(side, t, np.inf)
        tt = np.minimum(tt, np.where(cap, tc, np.inf))
        best = np.minimum(best, tt)
    return best


def _scan(sensor, yaw, boxes, cyls, rng_noise, rings=64, azimuths=1875, max_range=80.0,
          range_noise=0.02):
    elev = np.radians(np.linspace(-24.8, 2.0, rings))
    az = 2.0 * np.pi * np.arange(azimuths) / azimuths
    E, A = np.meshgrid(elev, az, indexing="ij")          # ring-major order
    d_loc = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)
    Rz = rotation_from_axis_angle([0, 0, 1], yaw)
    d = d_loc @ Rz.T
    t_ground = np.where(d[:, 2] < -1e-9, -sensor[2] / np.where(d[:, 2] < -1e-9, d[:, 2], -1.0), np.inf)
    t = np.minimum(t_ground, _ray_boxes(sensor, d, boxes))
    t = np.minimum(t, _ray_cylinders(sensor, d, cyls))
    keep = t <= max_range
    r = t[keep] + rng_noise.normal(0.0, range_noise, size=int(keep.sum()))
    return d_loc[keep] * r[:, None]


def _street(s_scene, sensors):
    """50 axis-aligned boxes (none over a sensor) and 30 upright cylinders."""
    boxes = []
    while len(boxes) < 50:
        side = s_scene.uniform(1.0, 10.0, size=3)
        rad = s_scene.uniform(5.0, 60.0)
        ang = s_scene.uniform(0.0, 2 * np.pi)
        c = np.array([rad * np.cos(ang), rad * np.sin(ang)])
        lo = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, 0.0])
        hi = np.array([c[0] + side[0] / 2, c[1] + side[1] / 2, side[2]])
        inside = any(np.all(sv[:2] >= lo[:2] - 0.5) and np.all(sv[:2] <= hi[:2] + 0.5) for sv in sensors)
        if not inside:
            boxes.append((lo, hi))
    cyls = []
    for _ in range(30):
        rad = s_scene.uniform(3.0, 50.0)
        ang = s_scene.uniform(0.0, 2 * np.pi)
        cyls.append((rad * np.cos(ang), rad * np.sin(ang), s_scene.uniform(0.2, 1.0),
                     s_scene.uniform(2.0, 8.0)))
    return boxes, cyls


def lidar_pair(seed: int, rings: int = 64, azimuths: int = 1875) -> PairSample:
    """Two sweeps of a spinning scanner; frame 2 is 1 m forward with a small yaw."""
    s_scene, _, _, s_noise, s_pose = [
        np.random.Generator(np.random.PCG64(ss)) for ss in np.random.SeedSequence(seed).spawn(5)
    ]
    h = 1.8
    sensors = [np.array([0.0, 0.0, h]), np.array([1.0, 0.0, h])]
    boxes, cyls = _street(s_scene, sensors)
    yaw = math.radians(s_pose.uniform(-2.0, 2.0))
    src = _scan(sensors[0], 0.0, boxes, cyls, s_noise, rings, azimuths)
    tgt = _scan(sensors[1], yaw, boxes, cyls, s_noise, rings, azimuths)
    src32 = as_soa(src)
    return PairSample(src=src32, tgt=as_soa(tgt),
                      R_true=rotation_from_axis_angle([0, 0, 1], yaw), t_true=np.array([1.0, 0.0, 0.0]),
                      extent=_extent(src32),
                      meta=dict(kind="lidar", seed=seed, yaw_deg=math.degrees(yaw),
                                n_src=src.shape[0], n_tgt=tgt.shape[0]))


@dataclass
class SequenceSample:
    clouds: np.ndarray       # (3, sum N) float32, frame k at [offsets[k], offsets[k+1])
    offsets: np.ndarray      # (F+1,) int64
    R_abs: np.ndarray        # (F, 3, 3): frame-0 coordinates = R_abs[k] @ frame-k coordinates + t_abs[k]
    t_abs: np.ndarray        # (F, 3)
    meta: dict = field(default_factory=dict)


def lidar_sequence(seed: int, frames: int = 16, step_m: float = 1.0, max_turn_deg: float = 2.0,
                   rings: int = 64, azimuths: int = 1875) -> SequenceSample:
    """Sweeps of a spinning scanner driving down a street of one static scene
    (the boxes and cylinders of the LiDAR pair's scene, plus building fronts
    9-13 m to either side of the road): each frame moves step_m along the
    current heading, then turns by a yaw drawn from U(-max_turn_deg,
    max_turn_deg).  Points are in each sensor's own frame; R_abs, t_abs give
    every frame's pose in frame 0."""
    s_scene, _, _, s_noise, s_pose = [
        np.random.Generator(np.random.PCG64(ss)) for ss in np.random.SeedSequence(seed).spawn(5)
    ]
    h = 1.8
    yaws = np.zeros(frames)
    centres = np.zeros((frames, 3))
    centres[0] = [0.0, 0.0, h]
    for k in range(1, frames):
        heading = rotation_from_axis_angle([0, 0, 1], yaws[k - 1]) @ np.array([step_m, 0.0, 0.0])
        centres[k] = centres[k - 1] + heading
        yaws[k] = yaws[k - 1] + math.radians(s_pose.uniform(-max_turn_deg, max_turn_deg))
    boxes, cyls = _street(s_scene, list(centres))
    # building fronts lining the road on both sides (gaps between them)
    for k in range(frames):
        for side in (-1.0, 1.0):
            if s_scene.random() < 0.3:
                continue
            off = rotation_from_axis_angle([0, 0, 1], yaws[k]) @ np.array([0.0, side * s_scene.uniform(9.0, 13.0),
                                                                            0.0])
            half = np.array([s_scene.uniform(1.5, 3.0), s_scene.uniform(1.0, 2.0)])
            c = centres[k, :2] + off[:2]
            boxes.append((np.array([c[0] - half[0], c[1] - half[1], 0.0]),
                          np.array([c[0] + half[0], c[1] + half[1], s_scene.uniform(4.0, 15.0)])))
    clouds = [_scan(centres[k], yaws[k], boxes, cyls, s_noise, rings, azimuths) for k in range(frames)]
    offsets = np.concatenate([[0], np.cumsum([c.shape[0] for c in clouds])]).astype(np.int64)
    R_abs = np.stack([rotation_from_axis_angle([0, 0, 1], y) for y in yaws])
    t_abs = centres - centres[0]
    return SequenceSample(clouds=as_soa(np.concatenate(clouds, axis=0)), offsets=offsets, R_abs=R_abs,
                          t_abs=t_abs, meta=dict(kind="lidar_sequence", seed=seed, frames=frames,
                                                 yaw_deg=np.degrees(yaws).tolist()))


# --------------------------------------------------------------------------
# depth camera in a furnished room
# --------------------------------------------------------------------------

def _ray_room(o, d, room):
    W, D, H = room
    best = np.full(d.shape[0], np.inf)
    for axis, lim in ((0, 0.0), (0, W), (1, 0.0), (1, D), (2, 0.0), (2, H)):
        den = d[:, axis]
        t = (lim - o[axis]) / np.where(np.abs(den) < 1e-12, 1e-12, den)
        best = np.where((t > 1e-6) & (t < best), t, best)
    return best


def _ray_spheres(o, d, spheres):
    best = np.full(d.shape[0], np.inf)
    a = np.sum(d * d, axis=1)
    for c, r in spheres:
        oc = o - c
        b = 2 * d @ oc
        cc = oc @ oc - r * r
        disc = b * b - 4 * a * cc
        ok = disc >= 0
        t = (-b - np.sqrt(np.where(ok, disc, 0.0))) / (2 * a)
        best = np.where(ok & (t > 1e-6) & (t < best), t, best)
    return best


def _ray_yawed_boxes(o, d, boxes):
    best = np.full(d.shape[0], np.inf)
    for c, half, yaw in boxes:
        Rz = rotation_from_axis_angle([0, 0, 1], yaw)
        ol = Rz.T @ (o - c)
        dl = d @ Rz
        t = _ray_boxes(ol, dl, [(-half, half)])
        best = np.minimum(best, t)
    return best


def _render(cam_R, cam_c, room, boxes, spheres, rng_noise, rng_drop, width=640, height=480,
            f=525.0, drop=0.05):
    u, v = np.meshgrid(np.arange(width), np.arange(height), indexing="xy")
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    rays = np.stack([(u - cx) / f, (v - cy) / f, np.ones_like(u, dtype=np.float64)], -1).reshape(-1, 3)
    d = rays @ cam_R.T
    t = _ray_room(cam_c, d, room)
    t = np.minimum(t, _ray_yawed_boxes(cam_c, d, boxes))
    t = np.minimum(t, _ray_spheres(cam_c, d, spheres))
    valid = (t >= 0.5) & (t <= 4.0)
    z = t[valid]
    z = z + rng_noise.normal(0.0, 1.0, size=z.shape) * (0.0012 * z * z)
    pts = rays[valid] * z[:, None]
    keep = rng_drop.random(pts.shape[0]) >= drop
    return pts[keep]


def depth_pair(seed: int, width: int = 640, height: int = 480, downsample: int | None = None) -> PairSample:
    """Two depth-camera views of a room with boxes and spheres."""
    s_scene, s_src, s_tgt, s_noise, s_pose = [
        np.random.Generator(np.random.PCG64(ss)) for ss in np.random.SeedSequence(seed).spawn(5)
    ]
    room = (s_scene.uniform(3, 5), s_scene.uniform(3, 5), s_scene.uniform(2.5, 3.0))
    c1 = np.array([s_scene.uniform(1.0, room[0] - 1.0), s_scene.uniform(1.0, room[1] - 1.0), 1.5])
    yaw = s_scene.uniform(0, 2 * np.pi)
    pitch = math.radians(s_scene.uniform(-15, 15))
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    R1 = np.stack([right, down, fwd], axis=1)                # camera -> world
    axis = _unit_sphere(s_pose, 1)[0]
    RD = rotation_from_axis_angle(axis, math.radians(s_pose.uniform(0, 10)))
    tD = _unit_sphere(s_pose, 1)[0] * s_pose.uniform(0, 0.2)
    R2 = R1 @ RD
    c2 = c1 + R1 @ tD
    boxes, spheres = [], []
    while len(boxes) < 10:
        half = s_scene.uniform(0.2, 1.0, size=3) / 2
        c = np.array([s_scene.uniform(half.max(), room[0] - half.max()),
                      s_scene.uniform(half.max(), room[1] - half.max()), half[2]])
        if min(np.linalg.norm(c - c1), np.linalg.norm(c - c2)) > np.linalg.norm(half) + 0.6:
            boxes.append((c, half, s_scene.uniform(0, 2 * np.pi)))
    while len(spheres) < 10:
        r = s_scene.uniform(0.1, 0.5)
        c = np.array([s_scene.uniform(r, room[0] - r), s_scene.uniform(r, room[1] - r),
                      s_scene.uniform(r, room[2] - r)])
        if min(np.linalg.norm(c - c1), np.linalg.norm(c - c2)) > r + 0.6:
            spheres.append((c, r))
    src = _render(R1, c1, room, boxes, spheres, s_noise, s_src, width, height)
    tgt = _render(R2, c2, room, boxes, spheres, s_noise, s_tgt, width, height)
    if downsample is not None:
        src = src[np.sort(s_src.choice(src.shape[0], size=min(downsample, src.shape[0]), replace=False))]
        tgt = tgt[np.sort(s_tgt.choice(tgt.shape[0], size=min(downsample, tgt.shape[0]), replace=False))]
    src32 = as_soa(src)
    return PairSample(src=src32, tgt=as_soa(tgt), R_true=RD, t_true=tD, extent=_extent(src32),
                      meta=dict(kind="depth", seed=seed, n_src=src.shape[0], n_tgt=tgt.shape[0]))


# --------------------------------------------------------------------------
# uneven batch of small pairs
# --------------------------------------------------------------------------

def uneven_batch(seed_base: int = 3000, count: int = 256, n_min: int = 2_000, n_max: int = 200_000,
                 max_angle_deg: float = 45.0, leaf_points: float = 50.0) -> BatchSample:
    """``count`` planes+spheres pairs with N log-uniform in [n_min, n_max].

    The pair k uses seed ``seed_base + k``; its size comes from a separate
    stream ``SeedSequence((seed_base + k, 7))``.  Tree depth per pair is
    ceil(log8(N / leaf_points)).
    """
    srcs, tgts, Rs, ts, lv, ns = [], [], [], [], [], []
    for k in range(count):
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence((seed_base + k, 7))))
        nk = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        p = small_pair(seed_base + k, n=nk, max_angle_deg=max_angle_deg)
        srcs.append(p.src)
        tgts.append(p.tgt)
        Rs.append(p.R_true)
        ts.append(p.t_true)
        lv.append(max(1, int(math.ceil(math.log(nk / leaf_points, 8)))))
        ns.append(nk)
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    return BatchSample(src=np.ascontiguousarray(np.concatenate(srcs, axis=1)),
                       tgt=np.ascontiguousarray(np.concatenate(tgts, axis=1)),
                       src_offsets=off, tgt_offsets=off.copy(), levels=np.array(lv, dtype=np.int32),
                       R_true=np.stack(Rs), t_true=np.stack(ts),
                       meta=dict(kind="batch", seed_base=seed_base, count=count))


# --------------------------------------------------------------------------
# well-separated anisotropic blobs (exact-recovery fixtures)
# --------------------------------------------------------------------------

def blob_tree_cloud(seed: int, per_blob: int = 40, groups: int = 8, blobs_per_group: int = 8,
                    group_scale=(40.0, 25.0, 12.0), blob_scale=(4.0, 2.5, 1.2),
                    blob_sigma=(0.010, 0.006, 0.002)):
    """64 tight anisotropic blobs laid out as 8 groups of 8 around octant corners.

    Group centres sit at (+-a, +-b, +-c) with a > b > c, and inside each group
    the blobs sit at (+-a', +-b', +-c') about the group centre, so a PCA-octant
    split of the whole cloud and then of each group separates them.  Blob
    spreads are ~1e-2 against separations of several units, so the FP64
    responsibilities between blobs are exactly 0 or 1.
    Returns (xyz (3, M) float32, blob_id (M,), blob_centres (64, 3)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    signs = np.array([[1 if (k >> a) & 1 == 0 else -1 for a in range(3)] for k in range(8)], dtype=np.float64)
    pts, ids, centres = [], [], []
    bid = 0
    # random rotation of each blob's axes keeps the covariances anisotropic and generic
    for g in range(groups):
        gc = signs[g] * np.array(group_scale)
        for b in range(blobs_per_group):
            c = gc + signs[b] * np.array(blob_scale)
            q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
            local = rng.normal(size=(per_blob, 3)) * np.array(blob_sigma)
            pts.append(c + local @ q.T)
            ids.append(np.full(per_blob, bid))
            centres.append(c)
            bid += 1
    xyz = np.concatenate(pts)
    return as_soa(xyz), np.concatenate(ids), np.array(centres)
