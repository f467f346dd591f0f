"""The C-ABI library loads and exports every function include/ephx.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from helpers import header_symbols

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2002_02045_amd", "libephx.so")
HEADER = os.path.join(ROOT, "include", "ephx.h")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libephx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    syms = header_symbols(HEADER)
    assert len(syms) >= 18
    missing = [s for s in syms if not hasattr(lib, s)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="libephx.so not built")
def test_version_and_error_string_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.ephx_version.restype = ctypes.c_char_p
    lib.ephx_last_error.restype = ctypes.c_char_p
    assert lib.ephx_version().decode().startswith("ephx")
    # a null model is rejected before any device work
    lib.ephx_bands.restype = ctypes.c_int
    rc = lib.ephx_bands(None, 1, None, None, None, None, None)
    assert rc == -1
    assert "null" in lib.ephx_last_error().decode()
