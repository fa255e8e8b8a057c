"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_00095_amd", "libsnap.so")
HEADER = os.path.join(ROOT, "include", "snap.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snap_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("snap_plan_create", "snap_project", "snap_project_backward",
                     "snap_plan_destroy", "snap_plan_workspace_bytes"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.snap_error_string.restype = ctypes.c_char_p
    lib.snap_status_string.restype = ctypes.c_char_p
    assert lib.snap_error_string(-1) == b"invalid argument"
    assert lib.snap_status_string(0) == b"converged"
    lib.snap_plan_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.snap_plan_create(None, 0, None, None) == -1
