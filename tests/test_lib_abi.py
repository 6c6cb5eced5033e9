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


STRUCTS = {"Gaussians": "rgx_gaussians", "BuildOpts": "rgx_build_opts", "Camera": "rgx_camera",
           "RenderOpts": "rgx_render_opts", "Grads": "rgx_grads", "AdamGroup": "rgx_adam_group"}


def test_struct_layouts_match_the_header(tmp_path):
    """Every structure the binding passes through the boundary has the size
    and field offsets the header gives it (compiled by the host C compiler)."""
    import shutil
    import subprocess
    from paper_2509_07782_amd import lib
    hip_inc = "/opt/rocm/include"
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(hip_inc, "hip", "hip_runtime_api.h")):
        pytest.skip("no host C compiler or HIP headers")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rgx.h"', "int main(void) {"]
    expect = []
    for py, c in STRUCTS.items():
        cls = getattr(lib, py)
        lines.append(f'  printf("%zu\\n", sizeof({c}));')
        expect.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({c}, {name}));')
            expect.append(getattr(cls, name).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-I", hip_inc,
                    "-D__HIP_PLATFORM_AMD__", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == expect
