"""Host build of the device ray arithmetic against exact integer rounding
(tests/host/band_key_check.cpp): the band keys of the tile pass and the
signed distance of the other walks, over band walks of random rays with
frequent exact ties, at perturbed reciprocal estimates. CPU only: g++
compiles csrc/ray.hpp with its one inline-asm minimum replaced."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
RAY = os.path.join(HERE, "..", "paper_2310_05766_amd", "csrc", "ray.hpp")
ASM_MIN = '    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));\n'


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("rayhost")
    src = open(RAY).read()
    assert src.count(ASM_MIN) == 1, "the inline-asm minimum of ray.hpp changed"
    src = src.replace(ASM_MIN, "    r = a < b ? a : b;\n").replace("#include <hip/hip_runtime.h>", "")
    hpp = d / "ray_host.hpp"
    hpp.write_text(src)
    exe = d / "band_key_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", f'-DRAY_HPP="{hpp}"', "-o", str(exe),
                    os.path.join(HERE, "host", "band_key_check.cpp")], check=True)
    return str(exe)


@pytest.mark.parametrize("seed", [1, 2])
def test_band_keys_exact(checker, seed):
    out = subprocess.run([checker, str(seed), "20000"], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout
