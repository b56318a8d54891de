"""MI355X-native TSDF mapping (FeatSense, arXiv 2310.05766, Sec. VI).

Hand-written HIP kernels for gfx950 behind a C ABI (include/tsdf.h); this
package is the thin Python binding over it.
"""
from ._abi import TsdfError, LIB_PATH  # noqa: F401


def __getattr__(name):
    if name in ("TsdfMap", "integrate_batch"):
        from . import tsdf
        return getattr(tsdf, name)
    raise AttributeError(name)
