"""The C-ABI library loads and exports every entry point include/xlmimo.h
declares (no GPU call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xlmimo.h")
LIB = os.path.join(ROOT, "paper_2503_18118_amd", "libxlmimo.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xlmimo_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("xlmimo_gram_exact", "xlmimo_gram_closedform", "xlmimo_zf_mmse_sumrate",
                 "xlmimo_capacity_sweep", "xlmimo_ctx_create", "xlmimo_ctx_destroy"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    lib.xlmimo_version.restype = ctypes.c_char_p
    assert lib.xlmimo_version().startswith(b"xlmimo")


def test_binding_exports_match_header():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2503_18118_amd import xlmimo
    assert sorted(xlmimo.EXPORTED) == declared_symbols()


def test_null_context_is_rejected():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    for name in ("xlmimo_gram_exact", "xlmimo_gram_closedform", "xlmimo_zf_mmse_sumrate", "xlmimo_capacity_sweep"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
    assert lib.xlmimo_gram_exact(None, None, None, 0, None, None) == -1
    assert lib.xlmimo_ctx_destroy(None) == 0
