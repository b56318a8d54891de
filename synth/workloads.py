"""The five seeded workloads (map descriptors, scans, poses, arrival traces).

Each workload stands in for the paper's OS1-128 recordings (UOS Lab, UOS
Parking Lot, HILTI), which are not available: synthetic scans with the same
structured shape (rings x columns), the paper's voxel sizes and map extents,
ray-cast against seeded analytic scenes. Inputs only; no TSDF arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import scenes as S


@dataclass(frozen=True)
class MapSpec:
    dims: tuple          # window size in voxels (nx, ny, nz)
    origin: tuple        # global voxel index of the window's min corner
    voxel_size: float    # metres
    tau_u: int           # truncation, 1/1024-voxel units
    w_max: int           # weight cap

    @property
    def n_voxels(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


@dataclass
class Scan:
    xyz: np.ndarray      # float32 (n, 3), sensor frame, NaN = no return
    pose: np.ndarray     # float64 (4, 4) row-major world_T_sensor
    rings: int
    cols: int
    map_index: int = 0
    arrival_s: float = 0.0


@dataclass
class Workload:
    name: str
    maps: list
    scans: list = field(default_factory=list)
    extra: dict = field(default_factory=dict)


# -- config 1: one 16-beam scan of a room into a 128^3 map ------------------

def config1() -> Workload:
    scene = S.room_scene(1)
    pose = np.eye(4)
    xyz = S.scan(scene, pose, 16, 1024, (-15.0, 15.0), 0.01, (0.0, 30.0), 11)
    m = MapSpec((128, 128, 128), (-64, -64, -64), 0.05, 3072, 64)
    return Workload("plain 16x1024 scan -> 128^3 @ 5 cm", [m], [Scan(xyz, pose, 16, 1024)])


# -- config 2: OS1-128-shaped sequence into a fixed 512x512x256 map ---------

def config2_poses(n_scans: int = 50) -> list:
    g = S.rng(22)
    yaws = g.uniform(-2.0, 2.0, size=50)
    poses = []
    for k in range(n_scans):
        poses.append(S.pose_matrix((-24.5 + k, 0.0, 0.0), math.radians(yaws[k % 50])))
    return poses


def config2(n_scans: int = 50) -> Workload:
    scene = S.outdoor_scene(2)
    scans = []
    for k, pose in enumerate(config2_poses(n_scans)):
        xyz = S.scan(scene, pose, 128, 1024, (-22.5, 22.5), 0.02, (0.5, 60.0), 200 + k)
        scans.append(Scan(xyz, pose, 128, 1024))
    m = MapSpec((512, 512, 256), (-256, -256, -32), 0.064, 5120, 64)
    return Workload("OS1-128 128x1024 sequence -> 512x512x256 @ 6.4 cm", [m], scans)


# -- config 3: closed loop through a ring-buffer window ---------------------

LOOP_LENGTH_M = 300.0
LOOP_RADIUS_M = LOOP_LENGTH_M / (2.0 * math.pi)


def config3_poses(n_scans: int = 200) -> list:
    poses = []
    for k in range(n_scans):
        th = 2.0 * math.pi * k / 200.0
        pos = (LOOP_RADIUS_M * math.cos(th), LOOP_RADIUS_M * math.sin(th), 0.0)
        poses.append(S.pose_matrix(pos, th + math.pi / 2.0))
    return poses


def config3(n_scans: int = 200) -> Workload:
    scene = S.loop_scene(3, LOOP_RADIUS_M)
    scans = []
    for k, pose in enumerate(config3_poses(n_scans)):
        xyz = S.scan(scene, pose, 16, 1024, (-15.0, 15.0), 0.01, (0.0, 30.0), 300 + k)
        scans.append(Scan(xyz, pose, 16, 1024))
    # the window origin is placed by the recentre rule from the first pose;
    # the origin here is only a placeholder the caller overwrites.
    m = MapSpec((512, 512, 128), (0, 0, 0), 0.05, 3072, 64)
    return Workload("ring-buffer loop 16x1024 -> 512x512x128 @ 5 cm", [m], scans,
                    extra={"recentre_vox": 64, "chunk": 64})


# -- config 4: batched uneven scans into 16 maps ----------------------------

SHAPES4 = ((16, 512), (32, 1024), (64, 1024), (128, 1024), (128, 2048))


def config4_shapes(n_scans: int = 256) -> list:
    g = S.rng(4)
    idx = g.integers(0, len(SHAPES4), size=256)
    return [SHAPES4[i] for i in idx[:n_scans]]


def config4_scan(i: int, shape) -> Scan:
    rings, cols = shape
    fov = (-15.0, 15.0) if rings == 16 else (-22.5, 22.5)
    pose = S.random_room_pose(20000 + i)
    scene = S.room_scene(10000 + i, keep_clear=(tuple(pose[:3, 3]),))
    xyz = S.scan(scene, pose, rings, cols, fov, 0.01, (0.0, 30.0), (20000 + i, 1))
    return Scan(xyz, pose, rings, cols, map_index=i % 16)


def config4(n_scans: int = 256) -> Workload:
    shapes = config4_shapes(n_scans)
    scans = [config4_scan(i, shapes[i]) for i in range(n_scans)]
    maps = [MapSpec((256, 256, 256), (-128, -128, -128), 0.08, 5120, 64) for _ in range(16)]
    return Workload("batched uneven scans -> 16 x 256^3 @ 8 cm", maps, scans)


# -- config 5: serving sessions ---------------------------------------------

SIZES5 = ((256, 256, 256), (384, 384, 384), (512, 512, 256))


@dataclass
class Session:
    sid: int
    spec: MapSpec
    arrivals: np.ndarray   # seconds, increasing
    scene: S.Scene

    def scan(self, k: int) -> Scan:
        """Scan k of this session (generated on demand, deterministic)."""
        g = S.rng((50000 + self.sid, k))
        for _ in range(1000):
            pos = g.uniform(np.array([-3.5, -2.5, -1.0]), np.array([3.5, 2.5, 1.0]))
            if S.scene_clear_of(self.scene, pos):
                break
        yaw = g.uniform(0.0, 2 * np.pi)
        pose = S.pose_matrix(pos, yaw)
        noise_seed = (50000 + self.sid, k, 1)
        xyz = S.scan(self.scene, pose, 16, 1024, (-15.0, 15.0), 0.01, (0.0, 30.0), noise_seed)
        return Scan(xyz, pose, 16, 1024, map_index=self.sid, arrival_s=float(self.arrivals[k]))


def config5(n_sessions: int = 48, duration_s: float = 60.0, rate_hz: float = 10.0) -> list:
    g = S.rng(5)
    size_idx = g.integers(0, len(SIZES5), size=48)
    sessions = []
    for s in range(n_sessions):
        dims = SIZES5[size_idx[s]]
        origin = tuple(-d // 2 for d in dims)
        spec = MapSpec(dims, origin, 0.064, 5120, 64)
        ga = S.rng(40000 + s)
        t, arr = 0.0, []
        while True:
            t += ga.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            arr.append(t)
        sessions.append(Session(s, spec, np.array(arr), S.room_scene(30000 + s)))
    return sessions


# -- small randomised inputs for parity fuzzing -----------------------------

def fuzz_scan(seed, n_points: int, extent_m: float = 3.0, nan_frac: float = 0.05,
              grid_snap: float | None = None) -> np.ndarray:
    """Random float32 points in a cube of half-size extent_m, with a fraction
    of NaN returns; with grid_snap, coordinates are multiples of it (exact
    ties on voxel faces)."""
    g = S.rng(seed)
    pts = g.uniform(-extent_m, extent_m, size=(n_points, 3))
    if grid_snap:
        pts = np.round(pts / grid_snap) * grid_snap
    m = g.random(n_points) < nan_frac
    pts[m, g.integers(0, 3, size=int(m.sum()))] = np.nan
    return pts.astype(np.float32)


def fuzz_pose(seed, max_t: float = 1.0) -> np.ndarray:
    """Random rigid pose (rotation from a random unit quaternion)."""
    g = S.rng(seed)
    q = g.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    rot = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])
    m = np.eye(4)
    m[:3, :3] = rot
    m[:3, 3] = g.uniform(-max_t, max_t, size=3)
    return m
