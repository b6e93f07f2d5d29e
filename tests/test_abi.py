"""The C interface: every function that include/imf.h declares is exported by
libimf.so (loaded without calling into the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "imf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(imf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("imf_create", "imf_destroy", "imf_compute", "imf_submit", "imf_wait",
              "imf_cancel", "imf_query_footprint", "imf_tool_register", "imf_autotune",
              "imf_raster", "imf_fft_c2c", "imf_fft_r2c_3d", "imf_last_error", "imf_fft_size",
              "imf_heaviside", "imf_access_filter", "imf_plan_greedy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2002_07627_amd import library_path
    if not os.path.exists(library_path()):
        pytest.skip("libimf.so not built")
    lib = ctypes.CDLL(library_path())
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_fft_size_choice():
    from paper_2002_07627_amd import library_path, fft_size
    if not os.path.exists(library_path()):
        pytest.skip("libimf.so not built")
    for n in (2, 5, 100, 216, 375, 377, 500, 545, 1000):
        m = fft_size(n)
        assert n <= m <= 1024 and m % 2 == 0
        k = m
        for p in (2, 3, 5, 7):
            while k % p == 0:
                k //= p
        assert k == 1
    assert fft_size(1025) == -1


def test_python_binding_fails_loudly_without_library(monkeypatch):
    import paper_2002_07627_amd.imf as b
    monkeypatch.setattr(b, "_LIB_PATH", "/nonexistent/libimf.so")
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(ImportError):
        b.fft_size(10)
