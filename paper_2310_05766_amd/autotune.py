"""Autotuner of the integration's launch shape.

Tunes, for a given map shape and workload sample:
* the candidate-buffer tiling (tile edges 2^lt),
* the number of tile workgroups,
* the binning block size (points per block, one per thread: 128, 256, 512),
* the tile workgroup size (256 or 512 threads; a workgroup's key buffers
  grow with it).
The first two are searched together, then the block sizes for the best of
them. Every candidate runs the sample on a fresh map built on torch-owned
device memory and must leave a map bit-identical to the default
configuration's before it is timed; the arithmetic is the same for all of
them, only the work decomposition changes. Results are cached in a JSON file
keyed by the map and workload shape.
"""
from __future__ import annotations

import json
import os
import statistics
import time

from .tsdf import TsdfMap, integrate_batch

# (lt_x, lt_y, lt_z): 2^9..2^12 voxels per tile, z edge >= 8
TILINGS = [(3, 3, 3), (4, 4, 3), (3, 3, 4), (2, 3, 4), (4, 3, 3), (2, 2, 5), (3, 4, 4), (4, 4, 4)]
WORKGROUPS = [0, 1024, 4096]  # 0: as many as fit the device
BLOCKS = [(256, 256), (128, 256), (512, 256), (256, 512), (512, 512)]  # (binning block, tile workgroup)

DEFAULT = {"lt": (3, 3, 3), "workgroups": 0, "bin_block": 256, "tile_block": 256}


def _cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "tsdf_autotune.json")


def _key(spec, mode, sample):
    npts = sum(int(x.shape[0]) for x, _ in sample)
    return f"{tuple(spec.dims)}|vs={spec.voxel_size}|tau={spec.tau_u}|{mode}|scans={len(sample)}|pts={npts}"


class _Arrays:
    """Fresh device arrays of one map (torch tensors)."""

    def __init__(self, torch, spec):
        n = spec.n_voxels
        self.sdf = torch.zeros(n, dtype=torch.int16, device="cuda")
        self.w = torch.zeros(n, dtype=torch.int16, device="cuda")
        nb = TsdfMap.scratch_bytes(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
        self.scratch = torch.zeros((nb + 3) // 4, dtype=torch.int32, device="cuda")

    def zero(self):
        self.sdf.zero_()
        self.w.zero_()


def _run(m, sample, mode, stream):
    if mode == "batch":
        integrate_batch([(m, x, p) for x, p in sample], stream=stream)
    else:
        for x, p in sample:
            m.integrate(x, p)


def autotune(spec, sample, mode: str = "batch", reps: int = 3, use_cache: bool = True, log=None):
    """Best {"lt", "workgroups", "bin_block", "tile_block"} for integrating
    `sample` (list of (device xyz tensor, pose)) into a map of `spec`, as one
    batch (mode "batch") or scan by scan (mode "plain")."""
    import torch

    path = _cache_path()
    key = _key(spec, mode, sample)
    if use_cache and os.path.exists(path):
        try:
            cached = json.load(open(path)).get(key)
            if cached and "bin_block" in cached:
                return {"lt": tuple(cached["lt"]), "workgroups": cached["workgroups"],
                        "bin_block": cached["bin_block"], "tile_block": cached["tile_block"], "cached": True,
                        "ms": cached.get("ms")}
        except (OSError, ValueError):
            pass
    stream = torch.cuda.Stream()
    arrays = _Arrays(torch, spec)
    results = []
    ref = []

    def trial(lt, wg, blocks):
        arrays.zero()
        torch.cuda.synchronize()
        m = TsdfMap(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max, stream=stream,
                    arrays=(arrays.sdf, arrays.w, arrays.scratch))
        try:
            m.set_tiling(lt, wg)
            m.set_blocks(*blocks)
            _run(m, sample, mode, stream)
            m.synchronize()
            # every candidate must give the default configuration's map
            if not ref:
                ref.append((arrays.sdf.clone(), arrays.w.clone()))
            elif not (torch.equal(ref[0][0], arrays.sdf) and torch.equal(ref[0][1], arrays.w)):
                raise RuntimeError(f"tiling {lt} / {wg} workgroups / blocks {blocks} changed the map")
            times = []
            for _ in range(reps):
                m.synchronize()
                t0 = time.perf_counter()
                _run(m, sample, mode, stream)
                m.synchronize()
                times.append(time.perf_counter() - t0)
        finally:
            m.close()
        ms = 1e3 * statistics.median(times)
        results.append((ms, lt, wg, blocks))
        if log:
            log(f"autotune {mode}: lt={lt} workgroups={wg} blocks={blocks}: {ms:.3f} ms")
        return ms

    # tiling and workgroups at the default block sizes, then the block sizes
    for lt in TILINGS:
        for wg in WORKGROUPS:
            trial(lt, wg, BLOCKS[0])
    _, lt, wg, _ = min(results)
    for blocks in BLOCKS[1:]:
        trial(lt, wg, blocks)
    torch.cuda.synchronize()
    ms, lt, wg, blocks = min(results)
    best = {"lt": lt, "workgroups": wg, "bin_block": blocks[0], "tile_block": blocks[1], "ms": ms, "cached": False,
            "candidates": [{"lt": list(c[1]), "workgroups": c[2], "bin_block": c[3][0], "tile_block": c[3][1],
                            "ms": c[0]} for c in sorted(results)]}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            data = json.load(open(path)) if os.path.exists(path) else {}
            data[key] = {"lt": list(lt), "workgroups": wg, "bin_block": blocks[0], "tile_block": blocks[1], "ms": ms}
            with open(path + ".tmp", "w") as f:
                json.dump(data, f, indent=1)
            os.replace(path + ".tmp", path)
        except (OSError, ValueError):
            pass
    return best
