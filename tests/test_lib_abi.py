"""The C-ABI library loads on the CPU-only host and exports every symbol the
header declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rgx.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rgx_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("rgx_build_bvh", "rgx_render_forward", "rgx_render_backward", "rgx_create"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2509_07782_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    L = ctypes.CDLL(lib.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(lib.EXPORTS) == set(declared_symbols())


def test_status_strings_without_gpu():
    from paper_2509_07782_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("library not built")
    L = lib.load()
    assert L.rgx_status_string(0) == b"ok"
    assert L.rgx_status_string(-1) == b"invalid argument"
    # creating a context on a device that does not exist is an argument error
    h = ctypes.c_void_p()
    assert L.rgx_create(1 << 20, ctypes.byref(h)) == -1
