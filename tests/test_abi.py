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


def _oracle_and_product_sources():
    oracle_files = [f for f in glob.glob(os.path.join(ROOT, "oracle", "*")) if f.endswith((".c", ".h", ".py"))]
    product_files = [f for f in glob.glob(os.path.join(ROOT, "paper_2310_05766_amd", "**", "*"), recursive=True)
                     if os.path.isfile(f) and f.endswith((".hip", ".hpp", ".h", ".cpp", ".py"))]
    return oracle_files, product_files


def _strip_comments(txt):
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    txt = re.sub(r"//[^\n]*", "", txt)
    return txt


def _big_constants(files):
    """Integer literals of 2^16 or more, by value."""
    found = {}
    for f in files:
        txt = _strip_comments(open(f, errors="ignore").read())
        for m in re.finditer(r"\b(0[xX][0-9a-fA-F]+|\d{5,})[uUlL]*\b", txt):
            tok = m.group(1)
            v = int(tok, 16) if tok.lower().startswith("0x") else int(tok)
            if v >= 1 << 16:
                found.setdefault(v, set()).add(os.path.relpath(f, ROOT))
    return found


def test_oracle_and_library_share_no_constants():
    """No magic number (hash multipliers, mixing constants, tables) appears in
    both the oracle and the GPU library. Powers of two and all-ones masks
    (2^k, 2^k - 1) are limits and units of the method itself (2^20 units of
    Eq. (3), the 2^30 fixed-point range, 32-bit indices) and may appear in
    both."""
    oracle_files, product_files = _oracle_and_product_sources()
    a, b = _big_constants(oracle_files), _big_constants(product_files)

    def structural(v):
        return v & (v - 1) == 0 or (v + 1) & v == 0

    shared = {hex(v): (sorted(a[v]), sorted(b[v])) for v in set(a) & set(b) if not structural(v)}
    assert not shared, shared


def test_oracle_and_library_share_no_lines():
    """No non-trivial line of code (30 characters or more, whitespace
    normalised, comments dropped) appears in both the oracle's C source and
    the GPU library's sources."""
    oracle_files, product_files = _oracle_and_product_sources()

    def code_lines(files):
        out = {}
        for f in files:
            if not f.endswith((".c", ".h", ".hip", ".hpp", ".cpp")):
                continue
            for line in _strip_comments(open(f, errors="ignore").read()).splitlines():
                n = re.sub(r"\s+", " ", line.strip())
                if len(n) >= 30 and not n.startswith("#"):
                    out.setdefault(n, set()).add(os.path.relpath(f, ROOT))
        return out

    a, b = code_lines(oracle_files), code_lines(product_files)
    shared = {k: (sorted(a[k]), sorted(b[k])) for k in set(a) & set(b)}
    assert not shared, shared


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2310_05766_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _abi.lib()
