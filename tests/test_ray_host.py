"""Host builds of the device ray arithmetic (tests/host/*.cpp). CPU only:
g++ compiles csrc/ray.hpp with its one inline-asm minimum replaced.
* band_key_check: the band keys of the tile pass and the signed distance of
  the other walks against exact integer rounding, over band walks of random
  rays with frequent exact ties, at perturbed reciprocal estimates;
* box_walk_check: the tile pass's resumed box walks against the plain voxel
  walk;
* rdiv_check: the merge's exact division (Eq. (1)) against exact integer
  rounding, with perturbed reciprocal estimates;
* free_walk_check: carving's free-space walk, clipped to random boxes and to
  the carving scan's slabs, against the oracle's segment voxels and keys
  (the oracle is compiled with gcc and linked in)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
RAY = os.path.join(HERE, "..", "paper_2310_05766_amd", "csrc", "ray.hpp")
ASM_MIN = '    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));\n'


@pytest.fixture(scope="module")
def build(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("rayhost")
    src = open(RAY).read()
    assert src.count(ASM_MIN) == 1, "the inline-asm minimum of ray.hpp changed"
    src = src.replace(ASM_MIN, "    r = a < b ? a : b;\n").replace("#include <hip/hip_runtime.h>", "")
    hpp = d / "ray_host.hpp"
    hpp.write_text(src)

    def compile_check(name, with_oracle=False):
        exe = d / name
        extra = []
        if with_oracle:
            obj = d / "oracle.o"
            if not obj.exists():
                subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-c", "-o", str(obj),
                                os.path.join(HERE, "..", "oracle", "tsdf_oracle.c")], check=True)
            extra = [str(obj), "-lm"]
        subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", f'-DRAY_HPP="{hpp}"', "-o", str(exe),
                        os.path.join(HERE, "host", name + ".cpp"), *extra], check=True)
        return str(exe)

    return compile_check


@pytest.mark.parametrize("seed", [1, 2])
def test_band_keys_exact(build, seed):
    out = subprocess.run([build("band_key_check"), str(seed), "20000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout


@pytest.mark.parametrize("seed", [1, 2])
def test_tile_resume_matches_plain_walk(build, seed):
    """The tile pass's resumed box walks (crossing counts from the binning's
    tile walk, walk_advance, walk_enter_box, box_walk_from / box_walk_next)
    visit exactly the plain voxel walk's voxels of each tile, in order, with
    the same box index and distance numerator, over random rays, tilings and
    window clips."""
    out = subprocess.run([build("box_walk_check"), str(seed), "8000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout


@pytest.mark.parametrize("seed", [1, 2])
def test_free_walk_matches_oracle(build, seed):
    """Carving's free-space walk (LongWalk / FreeWalk) clipped to random boxes
    and to 8-voxel slabs of a window visits exactly the oracle's voxels of the
    segment [o, S] in that box, in order, with the oracle's keys; the slabs
    together give the segment's voxels in the window."""
    out = subprocess.run([build("free_walk_check", with_oracle=True), str(seed), "3000"], capture_output=True,
                         text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout


def test_merge_divisions_exact(build):
    """Eq. (1)'s division as the merges run it, exact against integer
    rounding."""
    out = subprocess.run([build("rdiv_check"), "5"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout
