"""Serving loop: many concurrent sensor sessions, each keeping its TSDF map
resident in device memory, with their scans integrated as they arrive by
continuous batching.

* Admission. A session is admitted when its map fits the memory budget next
  to the maps already resident; otherwise it waits (first come, first
  served) until closed sessions free memory.
* Lanes. Each session is bound to one of a few lanes (HIP streams). All of a
  session's scans run on its lane, so they merge in arrival order; batches
  on different lanes run concurrently on the device.
* Continuous batching. Every tick, each lane with a free slot takes the
  scans that have arrived, the head scans of every ready session (a few per
  session, in order), and launches them as one batch while earlier batches
  may still be on the device.
* Latency of a scan = completion of its batch (observed on the host) minus
  its arrival time.

The integration itself is the library's batched engine; the executor
interface lets the same scheduler drive a CPU stand-in in tests.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ScanRecord:
    sid: int
    k: int             # index of the scan within its session
    arrival: float     # seconds, server clock
    done: float = -1.0  # seconds, server clock
    stats: dict | None = None

    @property
    def latency(self):
        return self.done - self.arrival


class GpuExecutor:
    """Runs batches through the library on a few HIP streams."""

    def __init__(self, lanes: int = 2, stats: bool = False):
        import torch

        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]  # default priority
        self.want_stats = stats

    @staticmethod
    def map_bytes(spec, options=None) -> int:
        # int16 sdf + int16 weight per voxel; a map with carving or
        # interpolation also holds an 8-byte key per voxel
        return (12 if _key_volume(options) else 4) * spec.n_voxels

    def create_map(self, spec, lane: int, options=None):
        from .tsdf import TsdfMap

        m = TsdfMap.from_spec(spec, stream=self.streams[lane])
        apply_options(m, options)
        return m

    def launch(self, lane: int, items):
        """Enqueue [(map, xyz, pose), ...] on the lane; returns a token."""
        from .tsdf import integrate_batch

        st = self.streams[lane]
        stats = integrate_batch(items, stream=st, stats=self.want_stats)
        ev = self.torch.cuda.Event()
        ev.record(st)
        return ev, stats

    def done(self, token) -> bool:
        return token[0].query()

    def wait(self, token):
        token[0].synchronize()

    def token_stats(self, token):
        return token[1]

    def release_map(self, m):
        m.close()

    def close(self):
        from .tsdf import batch_release

        for st in self.streams:
            st.synchronize()
            batch_release(st)


def _key_volume(options) -> bool:
    return bool(options) and (bool(options.get("carving")) or options.get("interpolation") is not None)


def apply_options(m, options):
    """Per-session map options: {"carving": True} or {"interpolation":
    (vfov_deg, hlines)} (not both: the library rejects the pair)."""
    if not options:
        return
    unknown = set(options) - {"carving", "interpolation"}
    if unknown:
        raise ValueError(f"unknown map options {sorted(unknown)}")
    if options.get("interpolation") is not None:
        vfov, lines = options["interpolation"]
        m.set_interpolation(vfov, lines)
    if options.get("carving"):
        m.set_carving(True)


@dataclass
class _Session:
    sid: int
    spec: object
    lane: int
    bytes: int
    options: object = None
    map: object = None
    queue: collections.deque = field(default_factory=collections.deque)  # (k, xyz, pose, record)
    inflight: int = 0
    closing: bool = False
    closed: bool = False


class Server:
    def __init__(self, executor, budget_bytes: int, lanes: int = 2, max_batch: int = 64,
                 max_per_session: int = 4, inflight_per_lane: int = 2, clock=time.perf_counter,
                 on_release=None):
        self.ex = executor
        self.on_release = on_release  # called as on_release(sid, map) before a map is freed
        self.budget = int(budget_bytes)
        self.lanes = lanes
        self.max_batch = max_batch
        self.max_per_session = max_per_session
        self.inflight_per_lane = inflight_per_lane
        self.clock = clock
        self.t0 = clock()
        self.used = 0
        self.sessions: dict[int, _Session] = {}
        self.waiting: collections.deque = collections.deque()
        self.inflight = [collections.deque() for _ in range(lanes)]  # (token, [records])
        self.completed: list[ScanRecord] = []
        self.batches = 0
        self.admit_log: list[tuple[float, int]] = []

    def now(self) -> float:
        return self.clock() - self.t0

    # -- sessions ---------------------------------------------------------------
    def open_session(self, sid: int, spec, options=None):
        """options: per-session map options (apply_options); they count in
        the session's memory."""
        nb = self.ex.map_bytes(spec, options) if options else self.ex.map_bytes(spec)
        if nb > self.budget:
            raise ValueError(f"session {sid}: map of {nb} bytes exceeds the whole budget")
        s = _Session(sid, spec, lane=sid % self.lanes, bytes=nb, options=options)
        self.sessions[sid] = s
        self.waiting.append(s)
        self._admit()
        return s

    def admitted(self, sid: int) -> bool:
        return self.sessions[sid].map is not None

    def _admit(self):
        while self.waiting and self.used + self.waiting[0].bytes <= self.budget:
            s = self.waiting.popleft()
            if s.closed:
                continue
            s.map = self.ex.create_map(s.spec, s.lane, s.options) if s.options else \
                self.ex.create_map(s.spec, s.lane)
            self.used += s.bytes
            self.admit_log.append((self.now(), s.sid))

    def close_session(self, sid: int):
        """Close once every submitted scan has completed (memory is freed then)."""
        s = self.sessions[sid]
        s.closing = True
        self._maybe_release(s)

    def _maybe_release(self, s: _Session):
        if s.closing and not s.closed and not s.queue and s.inflight == 0:
            s.closed = True
            if s.map is not None:
                if self.on_release:
                    self.on_release(s.sid, s.map)
                self.ex.release_map(s.map)
                s.map = None
                self.used -= s.bytes
            self._admit()

    # -- scans ------------------------------------------------------------------
    def submit(self, sid: int, k: int, xyz, pose, arrival: float | None = None) -> ScanRecord:
        s = self.sessions[sid]
        if s.closing:
            raise ValueError(f"session {sid} is closing")
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3)) \
            if isinstance(xyz, np.ndarray) else xyz
        if not np.isfinite(np.asarray(pose, dtype=np.float64)[:3]).all():
            raise ValueError("pose rows 0..2 must be finite")
        rec = ScanRecord(sid, k, self.now() if arrival is None else arrival)
        s.queue.append((k, xyz, pose, rec))
        return rec

    def step(self):
        """One scheduler tick: retire finished batches, admit, launch."""
        self._poll()
        self._admit()
        for lane in range(self.lanes):
            if len(self.inflight[lane]) >= self.inflight_per_lane:
                continue
            items, recs = [], []
            for s in self.sessions.values():
                if s.lane != lane or s.map is None or not s.queue:
                    continue
                for _ in range(min(self.max_per_session, len(s.queue))):
                    if len(items) >= self.max_batch:
                        break
                    k, xyz, pose, rec = s.queue.popleft()
                    items.append((s.map, xyz, pose))
                    recs.append((s, rec))
                if len(items) >= self.max_batch:
                    break
            if not items:
                continue
            token = self.ex.launch(lane, items)
            for s, _ in recs:
                s.inflight += 1
            self.inflight[lane].append((token, recs))
            self.batches += 1

    def _poll(self):
        for lane in range(self.lanes):
            q = self.inflight[lane]
            while q and self.ex.done(q[0][0]):
                token, recs = q.popleft()
                t = self.now()
                st = self.ex.token_stats(token)
                for j, (s, rec) in enumerate(recs):
                    rec.done = t
                    if st is not None:
                        rec.stats = st[j]
                    s.inflight -= 1
                    self.completed.append(rec)
                for s, _ in recs:
                    self._maybe_release(s)

    def pending(self) -> int:
        return sum(len(s.queue) for s in self.sessions.values()) + sum(len(q) for q in self.inflight)

    def drain(self, timeout_s: float = 600.0):
        t_end = self.clock() + timeout_s
        while self.pending():
            self.step()
            if self.clock() > t_end:
                raise TimeoutError("serving queue did not drain")
            time.sleep(0.0002)


def replay(server: Server, sessions, scans_of, speedup: float = 1.0, close_at_end: bool = True):
    """Replay an arrival trace: sessions = [(sid, spec, arrivals[])] or
    [(sid, spec, arrivals[], options)], and scans_of(sid, k) -> (xyz, pose).
    Arrival times are divided by speedup. Returns the completed records."""
    events = []
    last_k = {}
    for sess in sessions:
        sid, spec, arrivals = sess[:3]
        server.open_session(sid, spec, sess[3] if len(sess) > 3 else None)
        last_k[sid] = len(arrivals) - 1
        for k, t in enumerate(arrivals):
            events.append((float(t) / speedup, sid, k))
    events.sort()
    i = 0
    while i < len(events) or server.pending():
        now = server.now()
        while i < len(events) and events[i][0] <= now:
            t, sid, k = events[i]
            xyz, pose = scans_of(sid, k)
            server.submit(sid, k, xyz, pose, arrival=t)
            if close_at_end and k == last_k[sid]:
                server.close_session(sid)
            i += 1
        server.step()
        if i < len(events) and not server.pending():
            # nothing to do until the next arrival
            time.sleep(max(0.0, min(events[i][0] - server.now(), 0.001)))
        else:
            time.sleep(0.0001)
    return server.completed


def latency_summary(records):
    lat = np.array([r.latency for r in records if r.done >= 0]) * 1e3
    if lat.size == 0:
        return {}
    return {"scans": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()), "mean_ms": float(lat.mean())}
