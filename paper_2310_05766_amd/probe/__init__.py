"""Benchmark-only measurement aid: the device's scattered 64-bit atomicMin
rate (libtsdf_probe.so, built from atomic_probe.hip beside this file). It is
not part of the TSDF library or its C ABI; only bench.py and its test use it."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsdf_probe.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.probe_atomic_min_rate.restype = C.c_int
        L.probe_atomic_min_rate.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                            C.POINTER(C.c_float)]
        _lib = L
    return _lib


def atomic_probe(keys, waves: int = 2048, per_lane: int = 128, pattern: int = 0, stream=None) -> float:
    """Milliseconds for waves * 64 * per_lane scattered 64-bit atomicMins on
    the int64 device tensor keys (overwritten); pattern 1 keeps them in its
    first 4 MiB."""
    import torch
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.dtype == torch.int64 and keys.is_contiguous()):
        raise TypeError("keys must be a contiguous int64 CUDA tensor")
    ms = C.c_float()
    sh = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    rc = lib().probe_atomic_min_rate(C.c_void_p(keys.data_ptr()), keys.numel(), int(waves), int(per_lane),
                                     int(pattern), sh, C.byref(ms))
    if rc == -1:
        raise ValueError("probe_atomic_min_rate: invalid arguments")
    if rc != 0:
        raise RuntimeError(f"probe_atomic_min_rate failed ({rc})")
    return float(ms.value)
