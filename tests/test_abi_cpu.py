"""C interface checks that need no GPU: the library loads, exports every symbol
declared in include/mm.h, and rejects invalid arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2406_16064_amd", "libmmx.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def mm():
    if not os.path.exists(LIB):
        pytest.fail("libmmx.so not built (run python -m paper_2406_16064_amd.build)")
    from paper_2406_16064_amd import mm as m
    return m


def test_exports_every_declared_symbol(mm):
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mm.EXPORTED)


def test_status_strings(mm):
    assert mm.status_string(0) == "ok"
    assert "argument" in mm.status_string(-1)
    assert "h_min" in mm.status_string(-5)


def test_invalid_arguments_rejected_before_hip(mm):
    lib = mm._lib
    out = ctypes.c_void_p()
    assert lib.mm_plan_create(ctypes.byref(out), None, 0, 31, 1, None) == mm.MM_E_ARG
    bad = [mm.Mesh(1, 4, 1, 1e-9, 1e-9, 1e-9),       # nx < 2
           mm.Mesh(8, 0, 1, 1e-9, 1e-9, 1e-9),       # ny < 1
           mm.Mesh(8, 8, 1, -1e-9, 1e-9, 1e-9),      # negative cell
           mm.Mesh(8, 8, 1, float("nan"), 1e-9, 1e-9),
           mm.Mesh(4096, 8, 1, 1e-9, 1e-9, 1e-9)]    # beyond the supported size
    # one instance's [3][N] array at 4 GiB or more (32-bit offsets in the kernels):
    # 1024 x 1024 x 256 cells in FP64 (6 GiB) and 1024^3 in FP32 (12 GiB)
    big = [(mm.Mesh(1024, 1024, 256, 1e-9, 1e-9, 1e-9), 1), (mm.Mesh(1024, 1024, 1024, 1e-9, 1e-9, 1e-9), 0)]
    for msh, prec in big:
        assert lib.mm_plan_create(ctypes.byref(out), ctypes.byref(msh), prec, 31, 1, None) == mm.MM_E_ARG
        assert b"4 GiB" in lib.mm_last_error()
    for msh in bad:
        assert lib.mm_plan_create(ctypes.byref(out), ctypes.byref(msh), 0, 31, 1, None) == mm.MM_E_ARG
        assert lib.mm_last_error()
    good = mm.Mesh(8, 8, 1, 1e-9, 1e-9, 1e-9)
    assert lib.mm_plan_create(ctypes.byref(out), ctypes.byref(good), 7, 31, 1, None) == mm.MM_E_ARG
    assert lib.mm_plan_create(ctypes.byref(out), ctypes.byref(good), 0, 2048, 1, None) == mm.MM_E_ARG
    assert lib.mm_plan_create(ctypes.byref(out), ctypes.byref(good), 0, 31, 0, None) == mm.MM_E_ARG
    assert lib.mm_effective_field(None, None, 1, None, None, None) == mm.MM_E_ARG
    assert lib.mm_plan_destroy(None) == mm.MM_E_ARG
    assert lib.mm_plan_set_cells(None, 0, None, None, None, None) == mm.MM_E_ARG
    assert lib.mm_plan_set_shapes(None, None) == mm.MM_E_ARG
    assert lib.mm_plan_shapes(None, None) == mm.MM_E_ARG
    assert lib.mm_plan_tune_padding(None, None, 1, None, None, 3, None, None) == mm.MM_E_ARG
    assert lib.mm_neb_run(None, None, None, 3, 1e5, 1e-14, 1, None, None) == mm.MM_E_ARG
    assert lib.mm_heun_run(None, None, 1, None, 1e-13, 1, None) == mm.MM_E_ARG
    assert lib.mm_sd_run(None, None, 1, None, 1, 1e-7, 1e-9, 1e-3, None, None) == mm.MM_E_ARG
    assert lib.mm_sd_run_noalloc(None, None, 1, None, 1, 1e-7, 1e-9, 1e-3, None, None) == mm.MM_E_ARG
    assert lib.mm_demag_tensor(ctypes.byref(bad[0]), None, 1, None, None) == mm.MM_E_ARG
