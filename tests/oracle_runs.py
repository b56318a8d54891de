"""Helpers that run the oracle over whole workloads for the parity tests,
optionally one map per worker process (each worker single-threaded)."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

import oracle
import synth


def pool_size() -> int:
    # a one-GPU test host may give a job as few as 16 cores; stay well inside that
    return max(1, min(8, (os.cpu_count() or 2) - 1))


def run_map_sequence(spec, scans, origin=None):
    """Integrate scans in order into one oracle map; returns (sdf, w, stats)
    with sdf/w the window box in global C order [x][y][z]."""
    o = spec.origin if origin is None else origin
    m = oracle.OracleMap.from_spec(spec, origin=o)
    stats = [m.integrate(s.xyz, s.pose) for s in scans]
    sdf, w = m.readback(o, tuple(o[a] + spec.dims[a] for a in range(3)))
    m.close()
    return sdf, w, stats


def _config4_worker(args):
    map_index, n_scans = args
    shapes = synth.config4_shapes(n_scans)
    spec = synth.MapSpec((256, 256, 256), (-128, -128, -128), 0.08, 5120, 64)
    scans = [synth.config4_scan(i, shapes[i]) for i in range(n_scans) if i % 16 == map_index]
    sdf, w, stats = run_map_sequence(spec, scans)
    return map_index, sdf, w, stats


def config4_oracle(n_scans: int = 256, maps=range(16)):
    """Final window of each config-4 map (scan i -> map i mod 16), in parallel."""
    # fresh interpreters: the workers never share state with a process that
    # holds the GPU
    ctx = mp.get_context("spawn")
    with ctx.Pool(pool_size()) as pool:
        out = pool.map(_config4_worker, [(k, n_scans) for k in maps])
    return {k: (sdf, w, st) for k, sdf, w, st in out}


def _session_worker(args):
    sid, n_scans, n_sessions, duration = args
    sess = synth.config5(n_sessions=n_sessions, duration_s=duration)[sid]
    k_max = min(n_scans, len(sess.arrivals))
    scans = [sess.scan(k) for k in range(k_max)]
    sdf, w, stats = run_map_sequence(sess.spec, scans)
    return sid, sdf, w, stats


def sessions_oracle(sids, n_scans, n_sessions, duration):
    ctx = mp.get_context("spawn")
    with ctx.Pool(pool_size()) as pool:
        out = pool.map(_session_worker, [(s, n_scans, n_sessions, duration) for s in sids])
    return {s: (sdf, w, st) for s, sdf, w, st in out}


def window_digest(sdf: np.ndarray, w: np.ndarray) -> str:
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sdf).tobytes())
    h.update(np.ascontiguousarray(w).tobytes())
    return h.hexdigest()


def session_scans(args):
    """All scans of one config-5 session as stacked arrays (a worker job; no
    oracle call): (sid, xyz [n, 16384, 3] float32, poses [n, 4, 4])."""
    sid, n_sessions, duration = args
    sess = synth.config5(n_sessions=n_sessions, duration_s=duration)[sid]
    n = len(sess.arrivals)
    xyz = np.empty((n, 16 * 1024, 3), np.float32)
    poses = np.empty((n, 4, 4), np.float64)
    for k in range(n):
        sc = sess.scan(k)
        xyz[k] = sc.xyz
        poses[k] = sc.pose
    return sid, xyz, poses


def all_session_scans(n_sessions: int, duration: float):
    """Every scan of every config-5 session, generated in worker processes."""
    ctx = mp.get_context("spawn")
    workers = max(1, min(15, len(os.sched_getaffinity(0)) - 1))
    with ctx.Pool(workers) as pool:
        out = pool.map(session_scans, [(s, n_sessions, duration) for s in range(n_sessions)])
    return {sid: (x, p) for sid, x, p in out}


def load_digests():
    """The oracle's digests of the full-size workloads (written by
    tests/golden/make_oracle_digests.py, which calls only the oracle)."""
    import json
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")
    with open(path) as f:
        return json.load(f)


def input_digest(scans) -> str:
    import hashlib
    h = hashlib.sha256()
    for xyz, pose in scans:
        h.update(np.ascontiguousarray(xyz, dtype=np.float32).tobytes())
        h.update(np.ascontiguousarray(pose, dtype=np.float64).tobytes())
    return h.hexdigest()
