"""The C ABI library loads and exports every symbol include/grt.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grt.h")
LIB = os.path.join(ROOT, "paper_2607_22780_amd", "libgrt.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("grt_scene_build", "grt_trace", "grt_render_mis", "grt_render_mis_backward", "grt_trace_backward"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrt.so not built")
def test_binding_declares_every_symbol():
    from paper_2607_22780_amd import grt
    assert set(declared()) <= set(grt.SIGNATURES) | set(grt.OPTIONAL)
    lib = grt.load_library()
    assert lib.grt_version() >> 16 == 1
    assert lib.grt_status_str(-5).decode() == "GRT_ERR_ADMISSION"
    assert lib.grt_scene_workspace_bytes(1000) > 1000 * 64
    assert lib.grt_env_workspace_bytes(4, 8) > 0
    assert lib.grt_render_saved_bytes(10, 4) >= 640
    assert lib.grt_render_workspace_bytes(10, 4) >= 640
    assert lib.grt_trace_workspace_bytes(10) >= 64


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrt.so not built")
def test_host_argument_checks_without_gpu():
    """Argument validation happens on the host, before any device call."""
    from paper_2607_22780_amd import grt
    lib = grt.load_library()
    out = ctypes.c_void_p()
    assert lib.grt_scene_create(None, None, 0.0, None, 0, ctypes.byref(out)) == grt.ERR_INVALID
    assert lib.grt_trace(None, None, None, None, None, None, None, None, 0, None) == grt.ERR_INVALID
    assert b"scene" in lib.grt_last_error()
