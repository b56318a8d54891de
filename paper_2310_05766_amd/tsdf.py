"""Python face of the C ABI: one object per map, same call names.

Argument marshalling only -- every step of integration, shift and readback
runs in the HIP library. Host arrays are numpy; device arrays are torch
tensors (torch provides device memory and streams).
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _abi
from ._abi import check


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _pose_arg(pose):
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    return M, M.ctypes.data_as(C.POINTER(C.c_double))


_F32 = None


def _torch_float32():
    global _F32
    if _F32 is None:
        import torch

        _F32 = torch.float32
    return _F32


def _points_arg(xyz):
    """(pointer, n, kind, keepalive) for a numpy host array or a torch device tensor."""
    if isinstance(xyz, np.ndarray):
        a = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        return a.ctypes.data, a.shape[0], _abi.TSDF_PTR_HOST, a
    # torch tensor
    if xyz.dtype is not _torch_float32() or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
        raise ValueError("device points must be a contiguous float32 tensor of shape (n, 3)")
    if not xyz.is_cuda:
        a = xyz.numpy()
        return a.ctypes.data, a.shape[0], _abi.TSDF_PTR_HOST, a
    return xyz.data_ptr(), xyz.shape[0], _abi.TSDF_PTR_DEVICE, xyz


_ext_streams = {}
_order_events = {}
_recorded = {}  # id(tensor) -> (weak reference, torch streams it was recorded on)


def _record_once(t, ts):
    """t.record_stream(ts), once per tensor and stream: the allocator holds a
    recorded block until the stream has passed the point where the tensor is
    freed, which covers every later use on that stream too."""
    key = id(t)
    ent = _recorded.get(key)
    if ent is None or ent[0]() is not t:
        ent = _recorded[key] = (weakref.ref(t, lambda _r, k=key: _recorded.pop(k, None)), set())
    sid = ts.cuda_stream
    if sid not in ent[1]:
        t.record_stream(ts)
        ent[1].add(sid)


_held_by_stream = {}  # stream handle -> device tensors a caller-given raw stream may still read
_HOLD_MAX = 64


def _torch_stream(stream):
    """The torch stream object behind a stream argument, if it is one."""
    if stream is None or isinstance(stream, int):
        return None
    return stream


def _order_after_torch(handle):
    """The library's stream (handle) waits for torch's current stream, where
    the device points were written: a torch event recorded on the current
    stream, waited on by the library's stream. No-op for the same stream,
    and when the current stream has finished all its work already."""
    import torch

    cur = torch.cuda.current_stream()
    if handle is None or cur.cuda_stream == handle:
        return
    if cur.query():
        # everything torch's stream had queued is done, the points included:
        # nothing to wait for on the device
        return
    ext = _ext_streams.get(handle)
    if ext is None:
        ext = _ext_streams[handle] = torch.cuda.ExternalStream(handle)
    # one event per library stream, recorded again each time: a wait holds
    # the record it was queued after, so a later record cannot change it
    ev = _order_events.get(handle)
    if ev is None:
        ev = _order_events[handle] = torch.cuda.Event()
    ev.record(cur)
    ext.wait_event(ev)


def _hold_raw(handle, tensors):
    """Keep device points alive until a raw stream (one torch did not
    create) has read them: held here and released after that stream is
    synchronised (when the list grows long, or by _release_raw)."""
    held = _held_by_stream.setdefault(handle, [])
    if len(held) >= _HOLD_MAX:
        ext = _ext_streams.get(handle)
        if ext is not None:
            ext.synchronize()
        held.clear()
    held.extend(tensors)


def _release_raw(handle):
    _held_by_stream.pop(handle, None)


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # close maps while the HIP runtime is still up (interpreter-exit
    # finalisers may run after it is gone)
    for m in list(_live):
        try:
            m.close()
        except Exception:
            pass


class TsdfMap:
    """A TSDF window (int16 SDF + int16 weight per voxel) plus its host chunk store."""

    def __init__(self, dims, origin, voxel_size, tau_u, w_max, stream=None, arrays=None):
        self.desc = _abi.MapDesc((C.c_int32 * 3)(*[int(v) for v in dims]), (C.c_int32 * 3)(*[int(v) for v in origin]),
                                 float(voxel_size), int(tau_u), int(w_max))
        self.dims = tuple(int(v) for v in dims)
        self.voxel_size = float(voxel_size)
        self.tau_u, self.w_max = int(tau_u), int(w_max)
        self._h = C.c_void_p()
        self._keep = None
        L = _abi.lib()
        sh = _stream_handle(stream)
        # device points: a torch stream is told that the map reads them
        # (record_stream); the library's own stream gets a keep-alive list
        self._tstream = _torch_stream(stream)
        self._held = []
        if arrays is None:
            check(L.tsdf_map_create(C.byref(self.desc), sh, C.byref(self._h)), "tsdf_map_create")
        else:
            sdf, w, scratch = arrays  # caller-owned torch tensors
            self._keep = arrays
            check(L.tsdf_map_create_in(C.byref(self.desc), sdf.data_ptr(), w.data_ptr(), scratch.data_ptr(),
                                       scratch.numel() * scratch.element_size(), sh, C.byref(self._h)),
                  "tsdf_map_create_in")
        self._stream = self.device_arrays()[2]  # the map's HIP stream
        _live.add(self)

    @staticmethod
    def scratch_bytes(dims, origin, voxel_size, tau_u, w_max) -> int:
        d = _abi.MapDesc((C.c_int32 * 3)(*dims), (C.c_int32 * 3)(*origin), float(voxel_size), int(tau_u), int(w_max))
        return int(_abi.lib().tsdf_scratch_bytes(C.byref(d)))

    @classmethod
    def from_spec(cls, spec, origin=None, stream=None):
        return cls(spec.dims, spec.origin if origin is None else origin, spec.voxel_size, spec.tau_u, spec.w_max,
                   stream=stream)

    @property
    def handle(self):
        return self._h.value

    def close(self):
        if self._h:
            check(_abi.lib().tsdf_map_destroy(self._h), "tsdf_map_destroy")  # waits for the stream
            self._h = C.c_void_p()
            self._held = []
            _release_raw(self._stream)

    def _use(self, tensors):
        """Order device points for the map's stream and keep them alive until
        it has read them."""
        _order_after_torch(self._stream)
        if self._tstream is not None:
            for t in tensors:
                _record_once(t, self._tstream)
            return
        if len(self._held) >= _HOLD_MAX:
            self.synchronize()
        self._held.extend(tensors)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def integrate(self, xyz, pose, stats: bool = False):
        """tsdf_integrate_scan. With stats=True waits and returns the counts.
        Device points are read on the map's stream after torch's current
        stream has written them, and the map keeps them alive until its
        stream has read them, so the caller may drop them at once."""
        ptr, n, kind, _keep = _points_arg(xyz)
        if kind == _abi.TSDF_PTR_DEVICE:
            self._use([xyz])
        _M, Mp = _pose_arg(pose)
        st = _abi.ScanStats() if stats else None
        check(_abi.lib().tsdf_integrate_scan(self._h, ptr, n, kind, Mp, C.byref(st) if stats else None),
              "tsdf_integrate_scan")
        if stats:
            return dict(points_in=st.points_in, points_valid=st.points_valid, visits=st.visits,
                        voxels_updated=st.voxels_updated)
        return None

    def shift(self, new_origin):
        o = (C.c_int32 * 3)(*[int(v) for v in new_origin])
        check(_abi.lib().tsdf_shift(self._h, o), "tsdf_shift")

    def readback(self, lo, hi):
        lo_ = (C.c_int32 * 3)(*[int(v) for v in lo])
        hi_ = (C.c_int32 * 3)(*[int(v) for v in hi])
        shape = tuple(int(h) - int(l) for l, h in zip(lo, hi))
        sdf = np.zeros(shape, dtype=np.int16)
        w = np.zeros(shape, dtype=np.int16)
        check(_abi.lib().tsdf_readback(self._h, lo_, hi_, sdf.ctypes.data_as(C.POINTER(C.c_int16)),
                                       w.ctypes.data_as(C.POINTER(C.c_int16))), "tsdf_readback")
        return sdf, w

    def readback_window(self):
        o = self.origin
        return self.readback(o, tuple(o[a] + self.dims[a] for a in range(3)))

    @property
    def origin(self):
        o = (C.c_int32 * 3)()
        check(_abi.lib().tsdf_map_origin(self._h, o), "tsdf_map_origin")
        return tuple(int(v) for v in o)

    def device_arrays(self):
        s, w, st = C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(_abi.lib().tsdf_map_device_arrays(self._h, C.byref(s), C.byref(w), C.byref(st)),
              "tsdf_map_device_arrays")
        return s.value, w.value, st.value

    def recentre_origin(self, pose, radius_q10: int, chunk: int = 64, force: bool = False):
        _M, Mp = _pose_arg(pose)
        out = (C.c_int32 * 3)()
        due = C.c_int32(0)
        check(_abi.lib().tsdf_recentre_origin(self._h, Mp, int(radius_q10), int(chunk), int(bool(force)), out,
                                              C.byref(due)), "tsdf_recentre_origin")
        return bool(due.value), tuple(int(v) for v in out)

    def store_info(self):
        c, b = C.c_int64(), C.c_int64()
        check(_abi.lib().tsdf_store_info(self._h, C.byref(c), C.byref(b)), "tsdf_store_info")
        return int(c.value), int(b.value)

    def synchronize(self):
        check(_abi.lib().tsdf_map_synchronize(self._h), "tsdf_map_synchronize")
        self._held = []

    def register(self, xyz, init_pose, iterations: int = 10, damping: float = 1e-6):
        """Point-to-TSDF registration of a scan against this map: (pose,
        info) with info = points_used, cost, last_step, steps."""
        ptr, n, kind, keep = _points_arg(xyz)
        if kind == _abi.TSDF_PTR_DEVICE:
            self._use([xyz])
        M, Mp = _pose_arg(init_pose)
        out = np.zeros(16)
        info = _abi.RegisterInfo()
        check(_abi.lib().tsdf_register_scan(self._h, C.cast(ptr, C.POINTER(C.c_float)), n, kind, Mp,
                                            int(iterations), float(damping),
                                            out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(info)),
              "tsdf_register_scan")
        return out.reshape(4, 4), {"points": int(info.points_used), "cost": float(info.cost),
                                   "step": float(info.last_step), "steps": int(info.steps)}

    def register_sums(self, xyz, pose) -> np.ndarray:
        ptr, n, kind, keep = _points_arg(xyz)
        if kind == _abi.TSDF_PTR_DEVICE:
            self._use([xyz])
        M, Mp = _pose_arg(pose)
        out = np.zeros(29)
        check(_abi.lib().tsdf_register_sums(self._h, C.cast(ptr, C.POINTER(C.c_float)), n, kind, Mp,
                                            out.ctypes.data_as(C.POINTER(C.c_double))), "tsdf_register_sums")
        return out

    def mesh(self, lo, hi) -> np.ndarray:
        """Triangles (n, 3, 3) float32, metres, of the zero level set in the
        resident box [lo, hi) (marching tetrahedra, tsdf_mesh)."""
        lo_a, hi_a = (C.c_int32 * 3)(*[int(v) for v in lo]), (C.c_int32 * 3)(*[int(v) for v in hi])
        n = C.c_int64()
        check(_abi.lib().tsdf_mesh(self._h, lo_a, hi_a, None, 0, C.byref(n)), "tsdf_mesh")
        out = np.zeros((max(n.value, 1), 9), np.float32)
        check(_abi.lib().tsdf_mesh(self._h, lo_a, hi_a, out.ctypes.data_as(C.POINTER(C.c_float)), n.value,
                                   C.byref(n)), "tsdf_mesh")
        return out[:n.value].reshape(-1, 3, 3)

    def set_interpolation(self, vfov_deg: float = 0.0, hlines: int = 0):
        """Vertical interpolation between scan lines for the following scans
        (vfov in degrees over hlines scan lines; vfov 0 turns it off).
        Returns delta_z in 1/2^20 units."""
        check(_abi.lib().tsdf_map_set_interpolation(self._h, float(vfov_deg), int(hlines)),
              "tsdf_map_set_interpolation")
        return self.get_interpolation()

    def get_interpolation(self) -> int:
        d = C.c_int64()
        check(_abi.lib().tsdf_map_get_interpolation(self._h, C.byref(d)), "tsdf_map_get_interpolation")
        return int(d.value)

    def set_carving(self, on: bool = True) -> bool:
        """Free-space carving for the following scans: each ray longer than
        tau is also walked from the sensor to the start of its band."""
        check(_abi.lib().tsdf_map_set_carving(self._h, 1 if on else 0), "tsdf_map_set_carving")
        return self.get_carving()

    def get_carving(self) -> bool:
        v = C.c_int32()
        check(_abi.lib().tsdf_map_get_carving(self._h, C.byref(v)), "tsdf_map_get_carving")
        return bool(v.value)

    def key_atomics(self) -> int:
        """64-bit atomics the key-volume paths issued since the last call."""
        v = C.c_int64()
        check(_abi.lib().tsdf_map_key_atomics(self._h, C.byref(v)), "tsdf_map_key_atomics")
        return int(v.value)

    def set_tiling(self, log2_tile, workgroups: int = 0):
        """Candidate-buffer tiling (2^log2_tile voxels per axis); results do not depend on it."""
        lt = (C.c_int32 * 3)(*[int(v) for v in log2_tile])
        check(_abi.lib().tsdf_map_set_tiling(self._h, lt, int(workgroups)), "tsdf_map_set_tiling")

    def set_blocks(self, bin_block: int = 0, tile_block: int = 0):
        """Binning block size (128, 256, 512) and tile workgroup size (256,
        512); 0 selects the default. Results do not depend on them."""
        check(_abi.lib().tsdf_map_set_blocks(self._h, int(bin_block), int(tile_block)), "tsdf_map_set_blocks")

    def get_blocks(self):
        b, t = C.c_int32(), C.c_int32()
        check(_abi.lib().tsdf_map_get_blocks(self._h, C.byref(b), C.byref(t)), "tsdf_map_get_blocks")
        return int(b.value), int(t.value)

    def get_tiling(self):
        lt = (C.c_int32 * 3)()
        g = C.c_int32()
        check(_abi.lib().tsdf_map_get_tiling(self._h, lt, C.byref(g)), "tsdf_map_get_tiling")
        return tuple(int(v) for v in lt), int(g.value)

    def profile(self, on: bool = True):
        """Start (clearing earlier records) or stop per-kernel event timing."""
        check(_abi.lib().tsdf_profile_enable(self._h, int(bool(on))), "tsdf_profile_enable")

    def profile_read(self, kernel: str):
        """(total_ms, launches) of one kernel since profiling was enabled."""
        ms, n = C.c_double(), C.c_int64()
        check(_abi.lib().tsdf_profile_read(self._h, _abi.KERNELS[kernel], C.byref(ms), C.byref(n)),
              "tsdf_profile_read")
        return float(ms.value), int(n.value)


# numpy view of tsdf_scan_desc (map, xyz, n_points, pose[16])
_SCAN_DTYPE = np.dtype([("map", np.uint64), ("xyz", np.uint64), ("n", np.int64), ("pose", np.float64, (16,))])
assert _SCAN_DTYPE.itemsize == C.sizeof(_abi.ScanDesc)


def integrate_batch(items, stream=None, stats: bool = False):
    """tsdf_integrate_batch over [(TsdfMap, xyz, pose), ...]; scans sharing a
    map are applied in list order. All points must be of one kind. Device
    points are read on the batch's stream (stream, else the first map's)
    after torch's current stream has written them."""
    n = len(items)
    arr = np.zeros(max(n, 1), dtype=_SCAN_DTYPE)
    args = [_points_arg(xyz) for _, xyz, _ in items]
    keep = [a[3] for a in args]
    kinds = {a[2] for a in args}
    if n:
        # whole columns at once (per-element writes into a structured array
        # cost more than the launch itself for large batches)
        arr["map"][:n] = [m.handle for m, _, _ in items]
        arr["xyz"][:n] = [a[0] for a in args]
        arr["n"][:n] = [a[1] for a in args]
        arr["pose"][:n] = np.asarray([np.asarray(p, dtype=np.float64).reshape(16) for _, _, p in items])
    if len(kinds) > 1:
        raise ValueError("a batch takes host points or device points, not both")
    kind = kinds.pop() if kinds else _abi.TSDF_PTR_HOST
    if kind == _abi.TSDF_PTR_DEVICE and n > 0:
        tensors = [x for _, x, _ in items]
        if stream is None:
            items[0][0]._use(tensors)  # the batch runs on the first scan's map's stream
        else:
            handle = _stream_handle(stream)
            _order_after_torch(handle)
            ts = _torch_stream(stream)
            if ts is not None:
                for t in tensors:
                    _record_once(t, ts)
            else:
                _hold_raw(handle, tensors)
    st = (_abi.ScanStats * max(n, 1))() if stats else None
    check(_abi.lib().tsdf_integrate_batch(arr.ctypes.data_as(C.POINTER(_abi.ScanDesc)), n, kind,
                                          _stream_handle(stream), st), "tsdf_integrate_batch")
    if stats:
        return [dict(points_in=s.points_in, points_valid=s.points_valid, visits=s.visits,
                     voxels_updated=s.voxels_updated) for s in st[:n]]
    return None


def batch_release(stream):
    """Free the batch engine kept for a stream (call before destroying it)."""
    check(_abi.lib().tsdf_batch_release(_stream_handle(stream)), "tsdf_batch_release")  # waits for it
    _release_raw(_stream_handle(stream))


def set_graph_launch(on: bool):
    """Replay captured hipGraphs (default) or launch kernels directly."""
    check(_abi.lib().tsdf_set_graph_launch(int(bool(on))), "tsdf_set_graph_launch")


BATCH_STAGES = {"bin": 0, "tile": 1, "stats": 2, "launch": 3}


def batch_profile(stream, on: bool = True):
    """Per-stage event timing of the batch engine of a stream."""
    check(_abi.lib().tsdf_batch_profile(_stream_handle(stream), int(bool(on))), "tsdf_batch_profile")


def batch_profile_read(stream, stage: str):
    """(total_ms, launches) of one stage ("bin", "tile", "stats", "launch")."""
    ms, n = C.c_double(), C.c_int64()
    check(_abi.lib().tsdf_batch_profile_read(_stream_handle(stream), BATCH_STAGES[stage], C.byref(ms), C.byref(n)),
          "tsdf_batch_profile_read")
    return float(ms.value), int(n.value)
