"""Host-side checks of the boundary: the HIP library loads and exports every
function include/tsdf.h declares; the oracle and the GPU library share no
code. No GPU calls here."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsdf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsdf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tsdf_map_create", "tsdf_integrate_scan", "tsdf_shift", "tsdf_readback",
                     "tsdf_integrate_batch", "tsdf_map_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2310_05766_amd import _abi
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(_abi.EXPORTS)


def test_status_strings_without_gpu():
    from paper_2310_05766_amd import _abi
    assert _abi.status_string(0) == "ok"
    assert "invalid" in _abi.status_string(-1)


def test_oracle_and_library_share_no_code():
    product = glob.glob(os.path.join(ROOT, "paper_2310_05766_amd", "**", "*"), recursive=True)
    for f in product:
        if os.path.isfile(f) and f.endswith((".hip", ".hpp", ".h", ".py", ".cpp")):
            txt = open(f, errors="ignore").read()
            for bad in ("import oracle", "from oracle", "tsdf_oracle", "libtsdf_oracle"):
                assert bad not in txt, (f, bad)
    for f in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if f.endswith((".c", ".py", ".h")):
            txt = open(f).read()
            for bad in ("paper_2310_05766_amd", "tsdf.h", "ray.hpp", "libtsdf.so"):
                assert bad not in txt, (f, bad)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2310_05766_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _abi.lib()
