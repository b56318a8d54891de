#!/usr/bin/env python3
"""Writes tests/golden/oracle_digests.json: digests of the oracle's final maps
for the full-size workloads that are too slow to run beside every GPU test.

It calls only the CPU oracle (oracle/) and the seeded input generators
(synth/). Nothing here comes from the GPU library. The GPU parity tests and
the benchmark's serving leg compare the library's maps with these digests.

Entries:
  * config5: all 48 sessions over the full 60 s Poisson trace (about 28,800
    scans of 16x1024 points), one map per session, scans in arrival order;
  * carve50: free-space carving over the 50 OS1-128-shaped config-2 scans;
  * interp10: vertical interpolation (45 deg over 128 lines) over the first
    10 config-2 scans.
Each entry holds the sha256 of the final window (sdf bytes, then w bytes, C
order [x][y][z] over the window box), the per-scan counts (or their sums for
config 5), and a sha256 of the inputs (points and poses), so that a change of
the inputs is told apart from a parity failure.

Run from the repository root: python3 tests/golden/make_oracle_digests.py
(about 1,500 s of single-core oracle time, spread over worker processes).
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")


def window_digest(sdf, w) -> str:
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sdf).tobytes())
    h.update(np.ascontiguousarray(w).tobytes())
    return h.hexdigest()


def input_digest(scans) -> str:
    import numpy as np
    h = hashlib.sha256()
    for sc in scans:
        h.update(np.ascontiguousarray(sc.xyz, dtype=np.float32).tobytes())
        h.update(np.ascontiguousarray(sc.pose, dtype=np.float64).tobytes())
    return h.hexdigest()


def run(spec, scans, option=None):
    import oracle
    m = oracle.OracleMap.from_spec(spec)
    if option == "carving":
        m.set_carving(True)
    elif option == "interpolation":
        m.set_interpolation(45.0, 128)
    stats = [m.integrate(sc.xyz, sc.pose) for sc in scans]
    o = spec.origin
    sdf, w = m.readback(o, tuple(o[a] + spec.dims[a] for a in range(3)))
    m.close()
    return window_digest(sdf, w), stats


def session_job(sid):
    import synth
    sess = synth.config5(n_sessions=48, duration_s=60.0)[sid]
    scans = [sess.scan(k) for k in range(len(sess.arrivals))]
    dig, stats = run(sess.spec, scans)
    tot = {k: int(sum(s[k] for s in stats)) for k in ("points_valid", "visits", "voxels_updated")}
    return ("config5", sid, {"scans": len(scans), "window_sha256": dig, "inputs_sha256": input_digest(scans),
                             "dims": list(sess.spec.dims), "origin": list(sess.spec.origin), "totals": tot})


def config2_job(name):
    import synth
    n = 50 if name == "carve50" else 10
    wl = synth.config2(n)
    dig, stats = run(wl.maps[0], wl.scans, "carving" if name == "carve50" else "interpolation")
    per = [[int(s["points_valid"]), int(s["visits"]), int(s["voxels_updated"])] for s in stats]
    return (name, None, {"scans": n, "window_sha256": dig, "inputs_sha256": input_digest(wl.scans),
                         "per_scan_valid_visits_updated": per})


def job(arg):
    return config2_job(arg) if isinstance(arg, str) else session_job(arg)


def main():
    jobs = ["carve50", "interp10"] + list(range(48))
    out = {"config5": {}}
    workers = max(1, min(16, (os.cpu_count() or 2)))
    with mp.get_context("spawn").Pool(workers) as pool:
        for name, sid, rec in pool.imap_unordered(job, jobs):
            if name == "config5":
                out["config5"][str(sid)] = rec
            else:
                out[name] = rec
            print(name, sid, rec["window_sha256"][:16], flush=True)
    out["config5"] = {k: out["config5"][k] for k in sorted(out["config5"], key=int)}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
