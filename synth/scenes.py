"""Seeded synthetic LiDAR scenes and structured scans.

Input generation only: every function here returns float32 sensor-frame
points and float64 poses produced by ray casting analytic primitives in
float64. Nothing in this module computes any part of the TSDF method; the
oracle and the GPU path both consume its output unchanged.

Sensor model (a spinning multi-beam LiDAR, organised P x R scan: row = ring,
column = azimuth; paper Sec. II and Sec. III describe the structured layout):
  * ring k elevation e_k evenly spaced and inclusive over [e_min, e_max];
  * column j azimuth a_j = 2*pi*j/cols;
  * direction (cos e cos a, cos e sin a, sin e) in the sensor frame;
  * range = nearest positive hit + N(0, sigma^2);
  * a return outside the range gate, or with no hit, becomes NaN (no return).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_EPS = 1e-9


def rng(seed) -> np.random.Generator:
    """PCG64 generator for an integer seed or a sequence of integers."""
    if isinstance(seed, (list, tuple)):
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Scene:
    """Analytic scene. Every array is float64.

    room:      (lo[3], hi[3]) of an axis-aligned room seen from inside, or None
    ground:    (z, half_extent) of a square ground plane centred at the xy origin, or None
    spheres:   (k, 4)  centre xyz, radius
    boxes:     (k, 6)  lo xyz, hi xyz (axis aligned)
    cylinders: (k, 5)  centre x, centre y, radius, z_bottom, z_top (vertical)
    """

    room: tuple | None = None
    ground: tuple | None = None
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    cylinders: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))


def sensor_dirs(rings: int, cols: int, elev_min_deg: float, elev_max_deg: float) -> np.ndarray:
    """Unit ray directions in the sensor frame, ring-major: index = ring*cols + col."""
    if rings == 1:
        elev = np.array([math.radians(0.5 * (elev_min_deg + elev_max_deg))])
    else:
        k = np.arange(rings, dtype=np.float64)
        elev = np.radians(elev_min_deg + (elev_max_deg - elev_min_deg) * k / (rings - 1))
    az = 2.0 * np.pi * np.arange(cols, dtype=np.float64) / cols
    e = elev[:, None]
    a = az[None, :]
    d = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e) * np.ones_like(a)], axis=-1)
    return d.reshape(rings * cols, 3)


def pose_matrix(position, yaw: float = 0.0) -> np.ndarray:
    """4x4 row-major world_T_sensor for a yaw-only rotation and a translation."""
    c, s = math.cos(yaw), math.sin(yaw)
    m = np.eye(4, dtype=np.float64)
    m[0, 0], m[0, 1], m[1, 0], m[1, 1] = c, -s, s, c
    m[:3, 3] = np.asarray(position, dtype=np.float64)
    return m


# ---------------------------------------------------------------------------
# ray casting (float64, vectorised over rays)
# ---------------------------------------------------------------------------

def _hit_room_inside(p, d, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(d > 0, (hi - p) / d, np.where(d < 0, (lo - p) / d, np.inf))
    return t.min(axis=1)


def _hit_spheres(p, d, sph, t_best, idx):
    for cx, cy, cz, r in sph:
        sel = idx if idx is not None else slice(None)
        dd = d[sel]
        oc = p - np.array([cx, cy, cz])
        b = dd @ oc
        c2 = oc @ oc - r * r
        disc = b * b - c2
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t1 = -b - sq
        t2 = -b + sq
        t = np.where(t1 > _EPS, t1, np.where(t2 > _EPS, t2, np.inf))
        t = np.where(ok, t, np.inf)
        cur = t_best[sel]
        t_best[sel] = np.minimum(cur, t)


def _hit_aabb(p, dd, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dd
        t0 = (lo - p) * inv
        t1 = (hi - p) * inv
    t0 = np.nan_to_num(t0, nan=-np.inf)
    t1 = np.nan_to_num(t1, nan=np.inf)
    tmin = np.minimum(t0, t1).max(axis=1)
    tmax = np.maximum(t0, t1).min(axis=1)
    hit = tmax >= np.maximum(tmin, 0.0)
    t = np.where(tmin > _EPS, tmin, tmax)
    return np.where(hit & (t > _EPS), t, np.inf)


def _hit_cylinder(p, dd, cx, cy, r, z0, z1):
    ox, oy = p[0] - cx, p[1] - cy
    a = dd[:, 0] ** 2 + dd[:, 1] ** 2
    b = ox * dd[:, 0] + oy * dd[:, 1]
    c = ox * ox + oy * oy - r * r
    disc = b * b - a * c
    ok = (disc >= 0) & (a > 0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        ts = np.where(c < 0, (-b + sq) / a, (-b - sq) / a)
    zs = p[2] + ts * dd[:, 2]
    ts = np.where(ok & (ts > _EPS) & (zs >= z0) & (zs <= z1), ts, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        tc = np.where(dd[:, 2] != 0, (z1 - p[2]) / dd[:, 2], np.inf)
    hx = ox + tc * dd[:, 0]
    hy = oy + tc * dd[:, 1]
    tc = np.where((tc > _EPS) & (hx * hx + hy * hy <= r * r), tc, np.inf)
    return np.minimum(ts, tc)


class _AzimuthIndex:
    """Rays sorted by world azimuth, to test an object only against the rays
    whose horizontal direction can reach its bounding circle."""

    def __init__(self, d):
        self.az = np.arctan2(d[:, 1], d[:, 0])
        self.order = np.argsort(self.az, kind="stable")
        self.sorted = self.az[self.order]

    def select(self, p, cx, cy, rho):
        dx, dy = cx - p[0], cy - p[1]
        dist = math.hypot(dx, dy)
        if dist <= rho + 1e-6:
            return None  # sensor inside the bounding circle: every ray
        half = math.asin(min(1.0, rho / dist)) + 1e-6
        a0 = math.atan2(dy, dx)
        lo, hi = a0 - half, a0 + half
        parts = []
        for l, h in ((lo, hi), (lo + 2 * math.pi, hi + 2 * math.pi), (lo - 2 * math.pi, hi - 2 * math.pi)):
            i0 = np.searchsorted(self.sorted, max(l, -math.pi), side="left")
            i1 = np.searchsorted(self.sorted, min(h, math.pi), side="right")
            if i1 > i0:
                parts.append(self.order[i0:i1])
        if not parts:
            return np.zeros(0, dtype=np.int64)
        return np.concatenate(parts)


def cast(scene: Scene, origin, d_world: np.ndarray) -> np.ndarray:
    """Nearest positive hit distance for each ray (inf if none)."""
    p = np.asarray(origin, dtype=np.float64)
    n = d_world.shape[0]
    t_best = np.full(n, np.inf)
    if scene.room is not None:
        lo, hi = (np.asarray(v, dtype=np.float64) for v in scene.room)
        t_best = np.minimum(t_best, _hit_room_inside(p, d_world, lo, hi))
    if scene.ground is not None:
        zg, half = scene.ground
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(d_world[:, 2] != 0, (zg - p[2]) / d_world[:, 2], np.inf)
        hx = p[0] + t * d_world[:, 0]
        hy = p[1] + t * d_world[:, 1]
        t = np.where((t > _EPS) & (np.abs(hx) <= half) & (np.abs(hy) <= half), t, np.inf)
        t_best = np.minimum(t_best, t)
    index = _AzimuthIndex(d_world) if (len(scene.spheres) + len(scene.boxes) + len(scene.cylinders)) > 8 else None

    def rays_for(cx, cy, rho):
        if index is None:
            return None
        return index.select(p, cx, cy, rho)

    for cx, cy, cz, r in scene.spheres:
        sel = rays_for(cx, cy, r)
        _hit_spheres(p, d_world, np.array([[cx, cy, cz, r]]), t_best, sel)
    for b in scene.boxes:
        lo, hi = b[:3], b[3:]
        cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
        rho = 0.5 * math.hypot(hi[0] - lo[0], hi[1] - lo[1])
        sel = rays_for(cx, cy, rho)
        dd = d_world if sel is None else d_world[sel]
        t = _hit_aabb(p, dd, lo, hi)
        if sel is None:
            t_best = np.minimum(t_best, t)
        else:
            t_best[sel] = np.minimum(t_best[sel], t)
    for cx, cy, r, z0, z1 in scene.cylinders:
        sel = rays_for(cx, cy, r)
        dd = d_world if sel is None else d_world[sel]
        t = _hit_cylinder(p, dd, cx, cy, r, z0, z1)
        if sel is None:
            t_best = np.minimum(t_best, t)
        else:
            t_best[sel] = np.minimum(t_best[sel], t)
    return t_best


def scan(scene: Scene, pose: np.ndarray, rings: int, cols: int, elev_deg: tuple,
         sigma: float, range_gate: tuple, noise_seed) -> np.ndarray:
    """One structured scan: float32 (rings*cols, 3) sensor-frame points, NaN = no return."""
    d_s = sensor_dirs(rings, cols, elev_deg[0], elev_deg[1])
    rot = pose[:3, :3]
    d_w = d_s @ rot.T
    t = cast(scene, pose[:3, 3], d_w)
    noise = rng(noise_seed).normal(0.0, sigma, size=t.shape[0]) if sigma > 0 else np.zeros_like(t)
    rng_m = t + noise
    lo, hi = range_gate
    keep = np.isfinite(t) & (rng_m >= lo) & (rng_m <= hi) & (rng_m > 0)
    pts = d_s * np.where(keep, rng_m, 0.0)[:, None]
    pts[~keep] = np.nan
    return pts.astype(np.float32)


# ---------------------------------------------------------------------------
# scene recipes
# ---------------------------------------------------------------------------

def _dist_to_aabb(point, lo, hi):
    q = np.maximum(np.maximum(lo - point, 0.0), point - hi)
    return float(np.linalg.norm(q))


def room_scene(seed, room_lo=(-4.0, -3.0, -1.5), room_hi=(4.0, 3.0, 1.5), n_spheres=5, n_boxes=5,
               keep_clear=((0.0, 0.0, 0.0),), clearance=0.3) -> Scene:
    """Axis-aligned room seen from inside, with spheres r~U[0.2,0.8] m and
    axis-aligned boxes with sides U[0.3,1.5] m, centres uniform in the room.
    Objects closer than `clearance` to any point in `keep_clear` are redrawn."""
    g = rng(seed)
    lo = np.asarray(room_lo, dtype=np.float64)
    hi = np.asarray(room_hi, dtype=np.float64)
    clear = [np.asarray(c, dtype=np.float64) for c in keep_clear]
    spheres = []
    while len(spheres) < n_spheres:
        c = g.uniform(lo, hi)
        r = g.uniform(0.2, 0.8)
        if all(np.linalg.norm(c - k) - r >= clearance for k in clear):
            spheres.append([*c, r])
    boxes = []
    while len(boxes) < n_boxes:
        c = g.uniform(lo, hi)
        s = g.uniform(0.3, 1.5, size=3)
        blo, bhi = c - s / 2, c + s / 2
        if all(_dist_to_aabb(k, blo, bhi) >= clearance for k in clear):
            boxes.append([*blo, *bhi])
    return Scene(room=(lo, hi), spheres=np.array(spheres).reshape(-1, 4), boxes=np.array(boxes).reshape(-1, 6))


def loop_scene(seed, radius, n_spheres=300, n_boxes=300, band=10.0, clearance=0.5) -> Scene:
    """Room [-60,60]^2 x [-1.5,1.5] m enclosing a circular loop of the given
    radius at z = 0; spheres and boxes are placed within `band` metres of the
    loop and kept `clearance` metres away from the loop itself."""
    g = rng(seed)
    lo = np.array([-60.0, -60.0, -1.5])
    hi = np.array([60.0, 60.0, 1.5])

    def place():
        while True:
            ang = g.uniform(0.0, 2 * np.pi)
            rad = radius + g.uniform(-band, band)
            z = g.uniform(-1.5, 1.5)
            yield np.array([rad * math.cos(ang), rad * math.sin(ang), z])

    def dist_to_loop(pt_lo, pt_hi):
        # distance from the loop circle (z = 0) to an axis-aligned box, by
        # sampling the circle densely; enough for keeping objects clear.
        th = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
        pts = np.stack([radius * np.cos(th), radius * np.sin(th), np.zeros_like(th)], axis=1)
        q = np.maximum(np.maximum(pt_lo - pts, 0.0), pts - pt_hi)
        return float(np.sqrt((q * q).sum(axis=1)).min())

    spheres, boxes = [], []
    gen = place()
    while len(spheres) < n_spheres:
        c = next(gen)
        r = g.uniform(0.2, 0.8)
        if abs(math.hypot(c[0], c[1]) - radius) - r >= clearance or abs(c[2]) - r >= clearance:
            if dist_to_loop(c - r, c + r) >= clearance:
                spheres.append([*c, r])
    while len(boxes) < n_boxes:
        c = next(gen)
        s = g.uniform(0.3, 1.5, size=3)
        blo, bhi = c - s / 2, c + s / 2
        if dist_to_loop(blo, bhi) >= clearance:
            boxes.append([*blo, *bhi])
    return Scene(room=(lo, hi), spheres=np.array(spheres), boxes=np.array(boxes))


def outdoor_scene(seed, ground_z=-1.8, half=30.0, n_boxes=40, n_cyl=200, corridor_half=2.0) -> Scene:
    """Square ground plane, axis-aligned buildings (footprint sides U[2,10] m,
    height U[3,15] m) and vertical cylinders (r U[0.1,0.5] m, h U[2,8] m)
    standing on it, placed uniformly; none reaches into the corridor |y| <
    corridor_half around the driving line y = 0."""
    g = rng(seed)
    boxes = []
    while len(boxes) < n_boxes:
        fx, fy = g.uniform(2.0, 10.0, size=2)
        h = g.uniform(3.0, 15.0)
        cx, cy = g.uniform(-half, half, size=2)
        blo = np.array([cx - fx / 2, cy - fy / 2, ground_z])
        bhi = np.array([cx + fx / 2, cy + fy / 2, ground_z + h])
        if bhi[1] < -corridor_half or blo[1] > corridor_half:
            boxes.append([*blo, *bhi])
    cyl = []
    while len(cyl) < n_cyl:
        r = g.uniform(0.1, 0.5)
        h = g.uniform(2.0, 8.0)
        cx, cy = g.uniform(-half, half, size=2)
        if abs(cy) - r > corridor_half:
            cyl.append([cx, cy, r, ground_z, ground_z + h])
    return Scene(ground=(ground_z, half), boxes=np.array(boxes), cylinders=np.array(cyl))


def random_room_pose(seed, room_lo=(-4.0, -3.0, -1.5), room_hi=(4.0, 3.0, 1.5), shrink=0.5) -> np.ndarray:
    """Position uniform in the room shrunk by `shrink` metres, yaw U[0, 2pi)."""
    g = rng(seed)
    lo = np.asarray(room_lo) + shrink
    hi = np.asarray(room_hi) - shrink
    pos = g.uniform(lo, hi)
    yaw = g.uniform(0.0, 2 * np.pi)
    return pose_matrix(pos, yaw)


def scene_clear_of(scene: Scene, point, clearance=0.3) -> bool:
    pt = np.asarray(point, dtype=np.float64)
    for cx, cy, cz, r in scene.spheres:
        if np.linalg.norm(pt - np.array([cx, cy, cz])) - r < clearance:
            return False
    for b in scene.boxes:
        if _dist_to_aabb(pt, b[:3], b[3:]) < clearance:
            return False
    return True
