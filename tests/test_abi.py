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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_plan_queries_reject_null_plan_without_gpu():
    lib = ctypes.CDLL(LIB)
    i32 = ctypes.c_int32
    lib.snap_plan_describe.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.snap_plan_group_classes.argtypes = [ctypes.c_void_p, i32, ctypes.c_void_p, i32, ctypes.c_void_p]
    lib.snap_plan_set_group_class.argtypes = [ctypes.c_void_p, i32, i32]
    lib.snap_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.snap_project.argtypes = [ctypes.c_void_p] * 8
    lib.snap_project_backward.argtypes = [ctypes.c_void_p] * 9
    assert lib.snap_plan_describe(None, None, 0, None) == -1
    assert lib.snap_plan_group_classes(None, 0, None, 0, None) == -1
    assert lib.snap_plan_set_group_class(None, 0, 0) == -1
    assert lib.snap_plan_destroy(None) == -1
    assert lib.snap_project(*([None] * 8)) == -1
    assert lib.snap_project_backward(*([None] * 9)) == -1


class _Opt(ctypes.Structure):
    _fields_ = [("tol_h", ctypes.c_double), ("tol_s", ctypes.c_double), ("max_newton", ctypes.c_int32),
                ("max_ls", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_and_struct_sizes():
    lib = ctypes.CDLL(LIB)
    o = _Opt()
    lib.snap_default_options(ctypes.byref(o))
    assert (o.tol_h, o.tol_s, o.max_newton, o.max_ls, o.precision, o.flags) == (1e-11, 1e-11, 20, 30, 0, 0)
    # the structs the binding marshals have the header's layout
    from paper_2607_00095_amd import api
    assert ctypes.sizeof(api._Desc) == 72
    assert ctypes.sizeof(api._Opt) == 32
    assert api.STATS_DTYPE.itemsize == 32
