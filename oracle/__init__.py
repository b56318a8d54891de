"""TSDF oracle -- TEST INFRASTRUCTURE ONLY.

ctypes front end to the plain single-threaded C oracle in tsdf_oracle.c
(FeatSense, arXiv 2310.05766, Sec. VI). Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and this package never imports the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "tsdf_oracle.c")
LIB = os.path.join(_HERE, "libtsdf_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        L.or_rdiv.restype = C.c_int64
        L.or_rdiv.argtypes = [C.c_int64, C.c_int64]
        L.or_isqrt.restype = C.c_uint64
        L.or_isqrt.argtypes = [C.c_uint64]
        L.or_quantise_point.restype = C.c_int
        L.or_quantise_point.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_double), C.c_double, i64p]
        L.or_quantise_origin.restype = C.c_int
        L.or_quantise_origin.argtypes = [C.POINTER(C.c_double), C.c_double, i64p]
        L.or_band.restype = C.c_int
        L.or_band.argtypes = [i64p, i64p, C.c_int64, i64p, C.POINTER(C.c_uint64), i64p, i64p]
        L.or_segment_voxels.restype = C.c_int
        L.or_segment_voxels.argtypes = [i64p, i64p, i64p, C.c_int]
        L.or_voxel_sdf.restype = C.c_int64
        L.or_voxel_sdf.argtypes = [i64p, i64p, C.c_uint64, i64p, C.c_int64]
        L.or_key.restype = C.c_uint64
        L.or_key.argtypes = [C.c_int64, C.c_uint64]
        L.or_map_create.restype = C.c_void_p
        L.or_map_create.argtypes = [i32p, i32p, C.c_double, C.c_int32, C.c_int32]
        L.or_map_destroy.restype = None
        L.or_map_destroy.argtypes = [C.c_void_p]
        L.or_integrate.restype = C.c_int
        L.or_integrate.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_double), i64p]
        L.or_volume.restype = C.c_int
        L.or_volume.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_double), i64p,
                                C.POINTER(C.c_uint64)]
        L.or_shift.restype = C.c_int
        L.or_shift.argtypes = [C.c_void_p, i32p]
        L.or_readback.restype = C.c_int
        L.or_readback.argtypes = [C.c_void_p, i32p, i32p, C.POINTER(C.c_int16), C.POINTER(C.c_int16)]
        L.or_window.restype = C.c_int
        L.or_window.argtypes = [C.c_void_p, C.POINTER(C.c_int16), C.POINTER(C.c_int16), i32p]
        L.or_store_chunks.restype = C.c_int64
        L.or_store_chunks.argtypes = [C.c_void_p]
        L.or_interp_delta.restype = C.c_int64
        L.or_interp_delta.argtypes = [C.c_double, C.c_int32]
        L.or_up_vector.restype = None
        L.or_up_vector.argtypes = [C.POINTER(C.c_double), i64p]
        L.or_fill_offset.restype = None
        L.or_fill_offset.argtypes = [i64p, i64p, i64p, C.c_uint64, i64p, i64p, C.c_int64, i64p]
        L.or_set_interpolation.restype = C.c_int
        L.or_set_interpolation.argtypes = [C.c_void_p, C.c_int64]
        L.or_set_carving.restype = C.c_int
        L.or_set_carving.argtypes = [C.c_void_p, C.c_int]
        f64p = C.POINTER(C.c_double)
        L.or_reg_point.restype = C.c_int
        L.or_reg_point.argtypes = [C.c_void_p, C.POINTER(C.c_float), f64p, f64p, f64p, f64p]
        L.or_reg_sums.restype = C.c_int
        L.or_reg_sums.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64, f64p, f64p]
        L.or_reg_step.restype = C.c_int
        L.or_reg_step.argtypes = [f64p, C.c_double, f64p, f64p, f64p]
        L.or_register.restype = C.c_int
        L.or_register.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64, f64p, C.c_int32, C.c_double, f64p,
                                  f64p]
        L.or_set_voxels.restype = C.c_int
        L.or_set_voxels.argtypes = [C.c_void_p, i32p, i32p, C.POINTER(C.c_int16), C.POINTER(C.c_int16)]
        L.or_mesh.restype = C.c_int64
        L.or_mesh.argtypes = [C.c_void_p, i32p, i32p, C.POINTER(C.c_float), C.c_int64]
        L.or_recentre.restype = C.c_int
        L.or_recentre.argtypes = [i32p, i32p, C.c_double, C.POINTER(C.c_double), C.c_int64, C.c_int32,
                                  C.c_int, i32p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i32(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32))


def _i64(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int64))


# -- scalar helpers ---------------------------------------------------------

def rdiv(n: int, d: int) -> int:
    return int(lib().or_rdiv(int(n), int(d)))


def isqrt(n: int) -> int:
    return int(lib().or_isqrt(int(n)))


def quantise_point(p, pose, scale):
    q = np.zeros(3, dtype=np.int64)
    pp = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    ok = lib().or_quantise_point(_p(pp, C.c_float), _p(M, C.c_double), float(scale), _p(q, C.c_int64))
    return (q if ok else None)


def quantise_origin(pose, scale):
    o = np.zeros(3, dtype=np.int64)
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    ok = lib().or_quantise_origin(_p(M, C.c_double), float(scale), _p(o, C.c_int64))
    return (o if ok else None)


def band(q, o, tau_u):
    q, o = _i64(q), _i64(o)
    D = np.zeros(3, np.int64)
    S = np.zeros(3, np.int64)
    E = np.zeros(3, np.int64)
    r = C.c_uint64(0)
    ok = lib().or_band(_p(q, C.c_int64), _p(o, C.c_int64), int(tau_u), _p(D, C.c_int64), C.byref(r),
                       _p(S, C.c_int64), _p(E, C.c_int64))
    if not ok:
        return None
    return D, int(r.value), S, E


def segment_voxels(S, E, max_voxels: int = 4096) -> np.ndarray:
    S, E = _i64(S), _i64(E)
    out = np.zeros((max_voxels, 3), dtype=np.int64)
    n = lib().or_segment_voxels(_p(S, C.c_int64), _p(E, C.c_int64), _p(out, C.c_int64), max_voxels)
    if n < 0:
        raise ValueError("segment has more voxels than max_voxels")
    return out[:n].copy()


def voxel_sdf(q, D, r, g, tau_u) -> int:
    q, D, g = _i64(q), _i64(D), _i64(g)
    return int(lib().or_voxel_sdf(_p(q, C.c_int64), _p(D, C.c_int64), int(r), _p(g, C.c_int64), int(tau_u)))


def key(s: int, i: int) -> int:
    return int(lib().or_key(int(s), int(i)))


def interp_delta(vfov_deg: float, hlines: int) -> int:
    """Eq. (3) as a fixed-point integer (1/2^20 units)."""
    return int(lib().or_interp_delta(float(vfov_deg), int(hlines)))


def up_vector(pose):
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    U = _i64([0, 0, 0])
    lib().or_up_vector(_p(M, C.c_double), _p(U, C.c_int64))
    return tuple(int(v) for v in U)


def fill_offset(q, o, D, r, U, g, dq):
    """Offset e of the fill segment [c - e, c + e] of band voxel g."""
    e = _i64([0, 0, 0])
    args = [_i64(v) for v in (q, o, D)]
    Ua, ga = _i64(U), _i64(g)
    lib().or_fill_offset(*[_p(a, C.c_int64) for a in args], int(r), _p(Ua, C.c_int64), _p(ga, C.c_int64), int(dq),
                         _p(e, C.c_int64))
    return tuple(int(v) for v in e)


def reg_step(sums, lam, pose):
    """One damped Gauss-Newton step from normal-equation sums: (new pose, d)
    or None when the system is not positive definite."""
    S = np.ascontiguousarray(np.asarray(sums, dtype=np.float64))
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    out, d = np.zeros(16), np.zeros(6)
    if not lib().or_reg_step(_p(S, C.c_double), float(lam), _p(M, C.c_double), _p(out, C.c_double), _p(d, C.c_double)):
        return None
    return out.reshape(4, 4), d


def recentre(dims, origin, voxel_size, pose, radius_u, chunk=64, force=False):
    """(shift_due, new_origin) of the local-map recentre rule."""
    out = np.zeros(3, dtype=np.int32)
    d, o = _i32(dims), _i32(origin)
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    rc = lib().or_recentre(_p(d, C.c_int32), _p(o, C.c_int32), float(voxel_size), _p(M, C.c_double),
                           int(radius_u), int(chunk), int(bool(force)), _p(out, C.c_int32))
    if rc < 0:
        raise ValueError("pose not representable")
    return bool(rc), tuple(int(v) for v in out)


# -- the map ----------------------------------------------------------------

class OracleMap:
    """Window over the global TSDF volume plus the store of evicted voxels."""

    def __init__(self, dims, origin, voxel_size, tau_u, w_max):
        self.dims = tuple(int(v) for v in dims)
        self.voxel_size = float(voxel_size)
        self.tau_u, self.w_max = int(tau_u), int(w_max)
        d, o = _i32(dims), _i32(origin)
        self._m = lib().or_map_create(_p(d, C.c_int32), _p(o, C.c_int32), float(voxel_size), int(tau_u),
                                      int(w_max))
        if not self._m:
            raise ValueError("invalid map parameters or out of memory")

    @classmethod
    def from_spec(cls, spec, origin=None):
        return cls(spec.dims, spec.origin if origin is None else origin, spec.voxel_size, spec.tau_u, spec.w_max)

    def close(self):
        if self._m:
            lib().or_map_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_interpolation(self, vfov_deg: float = 0.0, hlines: int = 0, dq: int | None = None):
        """Vertical interpolation between scan lines for the following scans
        (vfov in degrees over hlines scan lines; vfov 0 turns it off)."""
        d = interp_delta(vfov_deg, hlines) if dq is None else int(dq)
        if lib().or_set_interpolation(self._m, d) != 0:
            raise ValueError("interpolation angle out of range")
        return d

    def set_carving(self, on: bool = True):
        """Free-space carving for the following scans: each ray is walked from
        the sensor to the end of its band (not with interpolation)."""
        if lib().or_set_carving(self._m, 1 if on else 0) != 0:
            raise ValueError("carving is not available together with interpolation")

    def integrate(self, xyz, pose) -> dict:
        x = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
        M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
        st = np.zeros(4, dtype=np.int64)
        rc = lib().or_integrate(self._m, _p(x, C.c_float), x.shape[0], _p(M, C.c_double), _p(st, C.c_int64))
        if rc != 0:
            raise ValueError(f"oracle integrate failed ({rc})")
        return dict(points_in=int(st[0]), points_valid=int(st[1]), visits=int(st[2]), voxels_updated=int(st[3]))

    def volume(self, xyz, pose, order=None) -> np.ndarray:
        """Per-scan candidate keys over the window in slot order (uint64).
        order: optional permutation of the rows, the order in which the
        points are taken (each keeps its row as its index)."""
        x = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
        M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
        out = np.empty(int(np.prod(self.dims)), dtype=np.uint64)
        op = None
        if order is not None:
            oa = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
            if oa.shape != (x.shape[0],):
                raise ValueError("order must hold one index per point")
            op = _p(oa, C.c_int64)
        rc = lib().or_volume(self._m, _p(x, C.c_float), x.shape[0], _p(M, C.c_double), op, _p(out, C.c_uint64))
        if rc != 0:
            raise ValueError(f"oracle volume failed ({rc})")
        return out.reshape(self.dims)

    def shift(self, new_origin):
        o = _i32(new_origin)
        rc = lib().or_shift(self._m, _p(o, C.c_int32))
        if rc != 0:
            raise ValueError(f"oracle shift failed ({rc})")

    def readback(self, lo, hi):
        lo_, hi_ = _i32(lo), _i32(hi)
        shape = tuple(int(h - l) for l, h in zip(lo_, hi_))
        sdf = np.zeros(shape, dtype=np.int16)
        w = np.zeros(shape, dtype=np.int16)
        rc = lib().or_readback(self._m, _p(lo_, C.c_int32), _p(hi_, C.c_int32), _p(sdf, C.c_int16),
                               _p(w, C.c_int16))
        if rc != 0:
            raise ValueError(f"oracle readback failed ({rc})")
        return sdf, w

    def window(self):
        """(sdf, w, origin) of the resident window in slot order."""
        sdf = np.zeros(self.dims, dtype=np.int16)
        w = np.zeros(self.dims, dtype=np.int16)
        o = np.zeros(3, dtype=np.int32)
        lib().or_window(self._m, _p(sdf, C.c_int16), _p(w, C.c_int16), _p(o, C.c_int32))
        return sdf, w, tuple(int(v) for v in o)

    def set_voxels(self, lo, hi, sdf, w):
        """Test helper: write a box of voxels (resident part only)."""
        lo, hi = _i32(lo), _i32(hi)
        s = np.ascontiguousarray(np.asarray(sdf, dtype=np.int16))
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.int16))
        lib().or_set_voxels(self._m, _p(lo, C.c_int32), _p(hi, C.c_int32), _p(s, C.c_int16), _p(ww, C.c_int16))

    def reg_point(self, p, pose):
        """(phi metres, gradient per metre, world point) or None."""
        pp = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
        phi, g, w = np.zeros(1), np.zeros(3), np.zeros(3)
        ok = lib().or_reg_point(self._m, _p(pp, C.c_float), _p(M, C.c_double), _p(phi, C.c_double),
                                _p(g, C.c_double), _p(w, C.c_double))
        return (float(phi[0]), g, w) if ok else None

    def reg_sums(self, xyz, pose) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
        M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
        out = np.zeros(29)
        lib().or_reg_sums(self._m, _p(x, C.c_float), x.shape[0], _p(M, C.c_double), _p(out, C.c_double))
        return out

    def register(self, xyz, pose0, iterations: int = 10, damping: float = 1e-6):
        """Damped Gauss-Newton point-to-TSDF registration: (pose, info) with
        info = points used, cost, last step norm, steps."""
        x = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32).reshape(-1, 3))
        M = np.ascontiguousarray(np.asarray(pose0, dtype=np.float64).reshape(16))
        out, info = np.zeros(16), np.zeros(4)
        lib().or_register(self._m, _p(x, C.c_float), x.shape[0], _p(M, C.c_double), int(iterations), float(damping),
                          _p(out, C.c_double), _p(info, C.c_double))
        return out.reshape(4, 4), {"points": int(info[0]), "cost": float(info[1]), "step": float(info[2]),
                                   "steps": int(info[3])}

    def mesh(self, lo, hi) -> np.ndarray:
        """Triangles (n, 3, 3) float32, metres, of the zero level set in the
        resident box [lo, hi) (marching tetrahedra)."""
        lo, hi = _i32(lo), _i32(hi)
        n = int(lib().or_mesh(self._m, _p(lo, C.c_int32), _p(hi, C.c_int32), None, 0))
        if n < 0:
            raise ValueError("box outside the window")
        out = np.zeros((max(n, 1), 9), np.float32)
        lib().or_mesh(self._m, _p(lo, C.c_int32), _p(hi, C.c_int32), _p(out, C.c_float), n)
        return out[:n].reshape(n, 3, 3)

    def store_chunks(self) -> int:
        return int(lib().or_store_chunks(self._m))
