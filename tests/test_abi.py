"""The C-ABI library loads and exports every entry point declared in
include/ftc.h; host-side argument checks work without a GPU (no kernel is
launched here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftc.h")
LIB = os.path.join(ROOT, "paper_2505_06932_amd", "libftc.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ftc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libftc.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_the_same_entry_points():
    from paper_2505_06932_amd import ftc
    assert sorted(ftc.EXPORTED) == _declared()


def test_status_strings(lib):
    lib.ftc_status_str.restype = C.c_char_p
    assert lib.ftc_status_str(0) == b"ok"
    assert b"margin" in lib.ftc_status_str(-2)
    assert lib.ftc_status_str(123) == b"unknown status"


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    from paper_2505_06932_amd import ftc
    f = lib.ftc_cells_create
    f.argtypes = [C.POINTER(C.c_void_p), C.POINTER(ftc._CGrid), C.c_int32, C.c_int32, C.c_int64, C.c_int32]
    f.restype = C.c_int32
    h = C.c_void_p()
    good = ftc._CGrid(16, 16, 16, 0.0, 0.0, 0.0, 1.0 / 16)
    assert f(None, C.byref(good), 10, 10, 100, 10) == ftc.FTC_EINVAL
    bad_h = ftc._CGrid(16, 16, 16, 0.0, 0.0, 0.0, 0.0)
    assert f(C.byref(h), C.byref(bad_h), 10, 10, 100, 10) == ftc.FTC_EINVAL
    small = ftc._CGrid(4, 16, 16, 0.0, 0.0, 0.0, 0.1)
    assert f(C.byref(h), C.byref(small), 10, 10, 100, 10) == ftc.FTC_EINVAL
    assert f(C.byref(h), C.byref(good), 0, 10, 100, 10) == ftc.FTC_EINVAL
    assert f(C.byref(h), C.byref(good), 10, 10, -1, 10) == ftc.FTC_EINVAL
    huge = ftc._CGrid(2000, 2000, 2000, 0.0, 0.0, 0.0, 1e-3)  # cell ids would overflow int32
    assert f(C.byref(h), C.byref(huge), 10, 10, 100, 10) == ftc.FTC_EINVAL
    assert h.value is None


def test_null_workspace_rejected(lib):
    from paper_2505_06932_amd import ftc
    g = ftc._CGrid(16, 16, 16, 0.0, 0.0, 0.0, 1.0 / 16)
    lib.ftc_build_cell_lists.restype = C.c_int32
    assert lib.ftc_build_cell_lists(None, C.byref(g), None, None) == ftc.FTC_EINVAL
    lib.ftc_last_device_error.restype = C.c_int32
    assert lib.ftc_last_device_error(None, None, None) == ftc.FTC_EINVAL
