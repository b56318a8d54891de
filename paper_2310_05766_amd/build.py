"""Build the HIP libraries (gfx950) in-tree: paper_2310_05766_amd/libtsdf.so
(the TSDF library) and paper_2310_05766_amd/probe/libtsdf_probe.so (the
benchmark's atomic-rate probe, a library of its own)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtsdf.so")
PROBE_SRC = os.path.join(HERE, "probe", "atomic_probe.hip")
PROBE_LIB = os.path.join(HERE, "probe", "libtsdf_probe.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # every float64 operation in the kernels is the one written (exact
    # integer arithmetic and the fixed fma chain of the transform)
    "-ffp-contract=off",
    "-fno-fast-math",
    # no packed-fp32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(os.path.dirname(HERE), "include"), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    ptmp = PROBE_LIB + ".tmp"
    pcmd = [hipcc, *HIPCC_FLAGS, "-o", ptmp, PROBE_SRC]
    if verbose:
        print(" ".join(pcmd), flush=True)
    subprocess.check_call(pcmd)
    os.replace(ptmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
