"""The C-ABI library loads, exports every function include/rc.h declares, and
rejects bad arguments on the host (no device work needed for these paths)."""
import ctypes
import os
import re

import paper_2602_03002_amd as m

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", text)))


def test_exports_match_header():
    names = declared_functions()
    assert "rc_render" in names and "rc_postprocess" in names
    lib = m.lib()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in rc.h but not exported"
    assert sorted(m.EXPORTED) == names


def test_host_validation_paths():
    L = m.lib()
    sz = ctypes.c_size_t()
    assert L.rc_scene_size(0, ctypes.byref(sz)) == -1
    assert L.rc_scene_size(1, None) == -1
    assert L.rc_scene_size(10, ctypes.byref(sz)) == 0 and sz.value > 0
    off = (ctypes.c_int64 * 3)(0, 5, 5)
    assert L.rc_robot_size(off, 2, ctypes.byref(sz)) == -1  # empty second link
    off = (ctypes.c_int64 * 3)(0, 5, 9)
    assert L.rc_robot_size(off, 2, ctypes.byref(sz)) == 0
    assert L.rc_robot_size(off, 65, ctypes.byref(sz)) == -1
    assert L.rc_render(None, None, None, 0, None) == -1
    assert L.rc_post_size(1, 1, 1, 1, -1, ctypes.byref(sz)) == -1
    assert L.rc_post_size(1, 2, 3, 4, 3, ctypes.byref(sz)) == 0 and sz.value >= 4 * 24 * 4
    assert L.rc_postprocess(None, None, None, None, 0, None, None, None, None, None) == -1
    assert L.rc_set_walk_stack_limit(None, 4) == -1
    assert b"NULL scene" in L.rc_last_error()
    assert L.rc_scene_destroy(None) == 0 and L.rc_post_destroy(None) == 0
    assert L.rc_status_string(-2) == b"workspace too small or misaligned"
    assert b"n_tri" in L.rc_last_error() or L.rc_last_error() != b""
