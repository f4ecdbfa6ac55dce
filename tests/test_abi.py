"""The C-ABI library loads and exports every function include/spx.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2006_14290_amd", "libspx.so")


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import sys
        sys.path.insert(0, ROOT)
        from paper_2006_14290_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for required in ("spx_spmv", "spx_csr_spmv", "spx_status_string", "spx_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version(lib):
    lib.spx_status_string.restype = ctypes.c_char_p
    lib.spx_status_string.argtypes = [ctypes.c_int]
    assert lib.spx_status_string(0) == b"SPX_OK"
    assert lib.spx_status_string(9) == b"SPX_ERR_ZERO_DIAG"
    assert lib.spx_status_string(99) == b"SPX_UNKNOWN"
    assert lib.spx_version() >= 100


def test_argument_errors_need_no_gpu(lib):
    # null descriptor and bad subwarp sizes are rejected on the host
    lib.spx_spmv.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double] * 2 + [ctypes.c_void_p]
    lib.spx_last_error.restype = ctypes.c_char_p
    assert lib.spx_spmv(None, None, None, 1.0, 0.0, None) == 1
    assert b"null" in lib.spx_last_error()
    lib.spx_subwarp_sum.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p]
    assert lib.spx_subwarp_sum(ctypes.c_void_p(16), ctypes.c_void_p(16), 64, 3, 1, None) == 1
    assert lib.spx_subwarp_sum(ctypes.c_void_p(16), ctypes.c_void_p(16), 65, 4, 1, None) == 1
