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


@pytest.mark.parametrize("compiler,lang", [("gcc", "c"), ("g++", "c++")])
def test_header_compiles_standalone(compiler, lang, tmp_path):
    """include/ftc.h is a plain C header (also valid C++): no HIP or torch types."""
    import subprocess
    src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
    src.write_text('#include "ftc.h"\nint main(void) { ftc_tuning t; (void)t; return (int)FTC_MLP_PARAMS - 6209; }\n')
    std = "-std=c99" if lang == "c" else "-std=c++14"
    r = subprocess.run([compiler, std, "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I",
                        os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_learned_and_tuning_entry_points_check_arguments_on_the_host(lib):
    """Null or out-of-range arguments are refused before any device work."""
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    lib.ftc_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
    lib.ftc_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp, i32, vp, vp]
    lib.ftc_mlp_loss_grad.argtypes = [vp, vp, C.c_int64, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.ftc_set_tuning.argtypes = [vp, vp]
    lib.ftc_get_tuning.argtypes = [vp, vp]
    EINVAL = -1
    assert lib.ftc_mlp_adam(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == EINVAL
    assert lib.ftc_mlp_forward(None, None, 10, None, None, 5, None, None) == EINVAL
    assert lib.ftc_mlp_loss_grad(None, None, 10, None, None, None, 5, None, None, None, None) == EINVAL
    assert lib.ftc_set_tuning(None, None) == EINVAL
    assert lib.ftc_get_tuning(None, None) == EINVAL
    # dummy non-null host pointers: the checks on step, rates and counts come first
    buf = (C.c_float * 8)()
    p = C.cast(buf, vp)
    assert lib.ftc_mlp_adam(p, p, p, p, 0, 1e-3, 0.9, 0.999, 1e-8, None) == EINVAL     # step counts from 1
    assert lib.ftc_mlp_adam(p, p, p, p, 1, -1.0, 0.9, 0.999, 1e-8, None) == EINVAL     # negative rate
    assert lib.ftc_mlp_adam(p, p, p, p, 1, 1e-3, 1.0, 0.999, 1e-8, None) == EINVAL     # beta1 = 1
    assert lib.ftc_mlp_loss_grad(p, p, 10, None, None, p, 0, p, None, p, None) == EINVAL  # empty batch
    assert lib.ftc_mlp_forward(p, p, 0, None, None, 5, p, None) == EINVAL                # no rows


def test_workspace_buffers_fit_the_registry():
    """Every device buffer a workspace allocates is registered for freeing in
    a fixed-size array: the allocations listed in the library source must
    not outnumber it (one more once wrote past it and crashed the destroy)."""
    with open(os.path.join(ROOT, "paper_2505_06932_amd", "csrc", "api.hip")) as f:
        src = f.read()
    cap = int(re.search(r"constexpr int kMaxBuffers = (\d+);", src).group(1))
    n = len(re.findall(r"^\s*FTC_ALLOC\(", src, flags=re.M))
    assert 0 < n <= cap, (n, cap)
