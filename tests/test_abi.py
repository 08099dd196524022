"""The C-ABI library loads and exports every entry point its header declares
(no compute: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2510_09081_amd import vrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrt.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vrt_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["vrt_create", "vrt_destroy", "vrt_voxelize", "vrt_cull", "vrt_trace", "vrt_frame_status",
              "vrt_query_as"]:
        assert f in fns
    assert set(fns) == set(vrt.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(vrt.LIB_PATH):
        pytest.fail("libvrt.so is not built (run paper_2510_09081_amd/build.py)")
    lib = ctypes.CDLL(vrt.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_status_strings_and_host_validation():
    L = vrt.load()
    assert L.vrt_status_string(0) == b"ok"
    assert b"capacity" in L.vrt_status_string(4)
    # host-side argument validation fails before touching a device
    assert L.vrt_create(None, None) == vrt.VRT_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    bad = vrt.vrt_desc(16, 16, 12, 0, 64, 0, 0)  # max_dim not a multiple of 8
    assert L.vrt_create(ctypes.byref(bad), ctypes.byref(h)) == vrt.VRT_ERR_INVALID_ARG
    assert L.vrt_voxelize(None, None, None, None) == vrt.VRT_ERR_INVALID_ARG
    assert L.vrt_copy_to_host(None, None, -1) == vrt.VRT_ERR_INVALID_ARG
    t = vrt.vrt_tune(256, 16, 4, 4, 4096)
    assert L.vrt_set_tune(None, 0, ctypes.byref(t)) == vrt.VRT_ERR_INVALID_ARG
    assert L.vrt_get_tune(None, 0, ctypes.byref(t)) == vrt.VRT_ERR_INVALID_ARG
    assert L.vrt_autotune(None, None, None, None) == vrt.VRT_ERR_INVALID_ARG
