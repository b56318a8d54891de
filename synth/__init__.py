"""Seeded synthetic inputs (scenes, scans, poses, arrival traces) shared by the
oracle tests and the GPU path. Holds no TSDF arithmetic."""
from .scenes import Scene, sensor_dirs, pose_matrix, scan, rng  # noqa: F401
from .workloads import (MapSpec, Scan, Workload, Session, config1, config2, config3,  # noqa: F401
                        config4, config5, config2_poses, config3_poses, config4_shapes,
                        config4_scan, fuzz_scan, fuzz_pose)
