"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/fruitninja.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fruitninja.h")
LIB = os.path.join(ROOT, "paper_2609_22608_amd", "libfruitninja.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_paths_calls():
    names = declared_functions()
    for n in ("fn_create", "fn_destroy", "fn_last_error", "plan_knn", "edge_time_batch",
              "edge_check", "risk_score"):
        assert n in names, n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.fn_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.fn_version()
    lib.fn_last_error.restype = ctypes.c_char_p
    assert lib.fn_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks_without_gpu():
    """NULL context / bad caps are rejected on the host before any HIP call."""
    lib = ctypes.CDLL(LIB)
    lib.fn_last_error.restype = ctypes.c_char_p
    rc = lib.plan_knn(None, None, ctypes.c_int64(4), 0, None, 1, 1, None, None, None)
    assert rc == -1 and b"NULL context" in lib.fn_last_error()
    from paper_2609_22608_amd import fn, workload as W
    d = fn.arm_desc(W.make_arm(0))
    d.n = 6
    caps = fn.Caps(16, 16, 4, 64)
    h = ctypes.c_void_p()
    lib.fn_create.argtypes = [ctypes.POINTER(fn.ArmDesc), ctypes.POINTER(fn.Caps),
                              ctypes.POINTER(ctypes.c_void_p)]
    assert lib.fn_create(ctypes.byref(d), ctypes.byref(caps), ctypes.byref(h)) == -3
    assert b"7 joints" in lib.fn_last_error()
