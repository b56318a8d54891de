"""ctypes declarations of the C ABI in include/tsdf.h (argument marshalling only).

The library must have been built (paper_2310_05766_amd/build.py); there is no
fallback: importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsdf.so")

TSDF_OK, TSDF_EINVAL, TSDF_ENOMEM, TSDF_EDEVICE, TSDF_ERANGE, TSDF_EBUSY = 0, -1, -2, -3, -4, -5
TSDF_PTR_HOST, TSDF_PTR_DEVICE = 0, 1

# every symbol include/tsdf.h declares
EXPORTS = (
    "tsdf_scratch_bytes", "tsdf_map_create", "tsdf_map_create_in", "tsdf_map_destroy", "tsdf_integrate_scan",
    "tsdf_shift", "tsdf_readback", "tsdf_integrate_batch", "tsdf_status_string", "tsdf_map_origin",
    "tsdf_map_device_arrays", "tsdf_recentre_origin", "tsdf_store_info", "tsdf_map_synchronize",
    "tsdf_profile_enable", "tsdf_profile_read", "tsdf_kernel_name", "tsdf_map_set_tiling",
    "tsdf_map_get_tiling", "tsdf_batch_release", "tsdf_set_graph_launch", "tsdf_batch_profile",
    "tsdf_batch_profile_read", "tsdf_map_set_interpolation", "tsdf_map_get_interpolation", "tsdf_mesh",
    "tsdf_register_scan", "tsdf_register_sums", "tsdf_map_set_carving", "tsdf_map_get_carving",
    "tsdf_map_key_atomics", "tsdf_integrate_scan_noalloc", "tsdf_map_set_blocks", "tsdf_map_get_blocks",
)
KERNELS = {"k_bin": 0, "k_tile": 1, "k_pack": 2, "k_unpack": 3}


class MapDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("origin", C.c_int32 * 3), ("voxel_size_m", C.c_double),
                ("tau_q10", C.c_int32), ("w_max", C.c_int32)]


class ScanStats(C.Structure):
    _fields_ = [("points_in", C.c_int64), ("points_valid", C.c_int64), ("visits", C.c_int64),
                ("voxels_updated", C.c_int64)]


class ScanDesc(C.Structure):
    _fields_ = [("map", C.c_void_p), ("xyz", C.c_void_p), ("n_points", C.c_int64), ("pose", C.c_double * 16)]


class RegisterInfo(C.Structure):
    _fields_ = [("points_used", C.c_int64), ("cost", C.c_double), ("last_step", C.c_double), ("steps", C.c_int32)]


class TsdfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run paper_2310_05766_amd/build.py)")
    # torch provides device memory and streams, so the process must hold one
    # HIP runtime: load torch's first; libtsdf.so's libamdhip64.so.7 then
    # resolves to the already-loaded copy instead of a second runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32p, i64 = C.c_void_p, C.POINTER(C.c_int32), C.c_int64
    st = C.c_int
    L.tsdf_scratch_bytes.restype = C.c_size_t
    L.tsdf_scratch_bytes.argtypes = [C.POINTER(MapDesc)]
    L.tsdf_map_create.restype = st
    L.tsdf_map_create.argtypes = [C.POINTER(MapDesc), vp, C.POINTER(vp)]
    L.tsdf_map_create_in.restype = st
    L.tsdf_map_create_in.argtypes = [C.POINTER(MapDesc), vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.tsdf_map_destroy.restype = st
    L.tsdf_map_destroy.argtypes = [vp]
    L.tsdf_integrate_scan.restype = st
    L.tsdf_integrate_scan.argtypes = [vp, vp, i64, C.c_int, C.POINTER(C.c_double), C.POINTER(ScanStats)]
    L.tsdf_shift.restype = st
    L.tsdf_shift.argtypes = [vp, i32p]
    L.tsdf_readback.restype = st
    L.tsdf_readback.argtypes = [vp, i32p, i32p, C.POINTER(C.c_int16), C.POINTER(C.c_int16)]
    f64p = C.POINTER(C.c_double)
    L.tsdf_register_scan.restype = st
    L.tsdf_register_scan.argtypes = [vp, C.POINTER(C.c_float), C.c_int64, C.c_int, f64p, C.c_int32, C.c_double, f64p,
                                     C.POINTER(RegisterInfo)]
    L.tsdf_register_sums.restype = st
    L.tsdf_register_sums.argtypes = [vp, C.POINTER(C.c_float), C.c_int64, C.c_int, f64p, f64p]
    L.tsdf_mesh.restype = st
    L.tsdf_mesh.argtypes = [vp, i32p, i32p, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_int64)]
    L.tsdf_map_set_interpolation.restype = st
    L.tsdf_map_set_interpolation.argtypes = [vp, C.c_double, C.c_int32]
    L.tsdf_map_get_interpolation.restype = st
    L.tsdf_map_get_interpolation.argtypes = [vp, C.POINTER(C.c_int64)]
    L.tsdf_map_set_carving.restype = st
    L.tsdf_map_set_carving.argtypes = [vp, C.c_int32]
    L.tsdf_map_get_carving.restype = st
    L.tsdf_map_get_carving.argtypes = [vp, C.POINTER(C.c_int32)]
    L.tsdf_integrate_scan_noalloc.restype = st
    L.tsdf_integrate_scan_noalloc.argtypes = [vp, vp, i64, C.POINTER(C.c_double), C.POINTER(ScanStats)]
    L.tsdf_map_set_blocks.restype = st
    L.tsdf_map_set_blocks.argtypes = [vp, C.c_int32, C.c_int32]
    L.tsdf_map_get_blocks.restype = st
    L.tsdf_map_get_blocks.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.tsdf_map_key_atomics.restype = st
    L.tsdf_map_key_atomics.argtypes = [vp, C.POINTER(C.c_int64)]
    L.tsdf_integrate_batch.restype = st
    L.tsdf_integrate_batch.argtypes = [C.POINTER(ScanDesc), C.c_int32, C.c_int, vp, C.POINTER(ScanStats)]
    L.tsdf_status_string.restype = C.c_char_p
    L.tsdf_status_string.argtypes = [C.c_int]
    L.tsdf_map_origin.restype = st
    L.tsdf_map_origin.argtypes = [vp, i32p]
    L.tsdf_map_device_arrays.restype = st
    L.tsdf_map_device_arrays.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
    L.tsdf_recentre_origin.restype = st
    L.tsdf_recentre_origin.argtypes = [vp, C.POINTER(C.c_double), i64, C.c_int32, C.c_int32, i32p, i32p]
    L.tsdf_store_info.restype = st
    L.tsdf_store_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.tsdf_map_synchronize.restype = st
    L.tsdf_map_synchronize.argtypes = [vp]
    L.tsdf_profile_enable.restype = st
    L.tsdf_profile_enable.argtypes = [vp, C.c_int32]
    L.tsdf_profile_read.restype = st
    L.tsdf_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.tsdf_map_set_tiling.restype = st
    L.tsdf_map_set_tiling.argtypes = [vp, i32p, C.c_int32]
    L.tsdf_map_get_tiling.restype = st
    L.tsdf_map_get_tiling.argtypes = [vp, i32p, C.POINTER(C.c_int32)]
    L.tsdf_batch_profile.restype = st
    L.tsdf_batch_profile.argtypes = [vp, C.c_int32]
    L.tsdf_batch_profile_read.restype = st
    L.tsdf_batch_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.tsdf_set_graph_launch.restype = st
    L.tsdf_set_graph_launch.argtypes = [C.c_int32]
    L.tsdf_batch_release.restype = st
    L.tsdf_batch_release.argtypes = [vp]
    L.tsdf_kernel_name.restype = C.c_char_p
    L.tsdf_kernel_name.argtypes = [C.c_int32]
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().tsdf_status_string(int(status)).decode()


def check(status: int, what: str):
    if status != TSDF_OK:
        raise TsdfError(status, what)
