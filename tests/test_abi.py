"""C-ABI checks that need no GPU: the library loads, exports every function that
include/vdamp.h declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_1911_01234_amd import vdamp as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "vdamp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_header_function():
    lib = V.load_library()
    names = header_functions()
    assert "vdamp_solve" in names and "fista_solve" in names and "vdamp_plan" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(V.EXPORTED)


def test_status_strings():
    lib = V.load_library()
    for code in range(8):
        assert lib.vdamp_status_string(code)
    assert lib.vdamp_status_string(99) == b"unknown status"


def _plan_status(batch, ny, nx, levels, wavelet=0, flags=0, null=None):
    lib = V.load_library()
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    a_ny = (ctypes.c_int32 * max(batch, 1))(*ny) if ny is not None else None
    a_nx = (ctypes.c_int32 * max(batch, 1))(*nx) if nx is not None else None
    st = lib.vdamp_plan(None if null == "plan" else ctypes.byref(h), batch, a_ny, a_nx, levels,
                        wavelet, flags, None if null == "ws" else ctypes.byref(wsb))
    return st, lib.vdamp_last_error().decode()


@pytest.mark.parametrize("args,code", [
    ((0, [64], [64], 3), 1),                 # empty batch
    ((1, [64], [64], 0), 3),                 # levels < 1
    ((1, [64], [64], 5), 3),                 # levels beyond this build
    ((1, [60], [64], 3), 2),                 # not divisible by 2^s
    ((1, [64], [1024], 3), 2),               # too large
    ((1, [64], [56], 3), 3),                 # 7 is not a supported radix
    ((2, [64, 64], [64, 4], 3), 2),          # second slice smaller than 2^s
    ((1, [64], [64], 3, 1), 3),              # unknown wavelet
    ((1, [64], [64], 3, 0, 1 << 30), 1),     # unknown flag
    ((1, [64], [48], 4), 3),                 # nx / 2^s odd: a coefficient pair would straddle two bands
])
def test_plan_rejects_bad_arguments(args, code):
    st, msg = _plan_status(*args)
    assert st == code, msg
    assert msg


def test_plan_null_pointers():
    assert _plan_status(1, [64], [64], 3, null="plan")[0] == 1
    assert _plan_status(1, [64], [64], 3, null="ws")[0] == 1
    assert _plan_status(1, None, [64], 3)[0] == 1


def test_solve_rejects_null_plan_and_workspace():
    lib = V.load_library()
    st = lib.vdamp_solve(None, None, None, 0, None, None, None, None, 1, None, None)
    assert st == 1
    st = lib.fista_solve(None, None, None, 0, None, None, None, 1, None, None)
    assert st == 1
    st = lib.vdamp_solve_resume(None, None, None, 0, None, None, None, None, None, None, None, None,
                                1, None, None, None)
    assert st == 1
    st = lib.vdamp_state_export(None, None, None, None, None, None, None, None)
    assert st == 1
    assert lib.vdamp_plan_destroy(None) == 1


def test_python_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(V, "_lib", None)
    monkeypatch.setattr(V, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        V.load_library()


def test_plan_accepts_512_slices():
    """512 x 512 with 4 levels: finest band of 65536 coefficients (the large-band search)
    passes every host check; without a GPU the plan then stops at its device upload."""
    lib = V.load_library()
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    n = (ctypes.c_int32 * 2)(512, 256)
    st = lib.vdamp_plan(ctypes.byref(h), 2, n, n, 4, 0, 0, ctypes.byref(wsb))
    msg = lib.vdamp_last_error().decode()
    if st == 0:
        assert lib.vdamp_plan_destroy(h) == 0
    else:
        assert st == 5 and "upload" in msg, msg


def test_plan_accepts_every_documented_flag():
    """All VDAMP_FLAG_* bits pass the host checks together (the autotune flag included);
    an undocumented bit is rejected before anything touches the device."""
    flags = (V.VDAMP_FLAG_DETERMINISTIC | V.VDAMP_FLAG_USE_GRAPH | V.VDAMP_FLAG_CHECK_FINITE
             | V.VDAMP_FLAG_TIMING | V.VDAMP_FLAG_AUTOTUNE | V.VDAMP_FLAG_SURE_CONTINUOUS
             | V.VDAMP_FLAG_GROUP_PAIRS)
    lib = V.load_library()
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    n = (ctypes.c_int32 * 1)(64)
    st = lib.vdamp_plan(ctypes.byref(h), 1, n, n, 3, 0, flags, ctypes.byref(wsb))
    msg = lib.vdamp_last_error().decode()
    if st == 0:
        assert lib.vdamp_plan_destroy(h) == 0
    else:
        assert st == 5 and "upload" in msg, msg
    st, msg = _plan_status(1, [64], [64], 3, 0, 1 << 9)
    assert st == 1 and "flag" in msg, msg


def test_describe_rejects_null_plan():
    lib = V.load_library()
    need = ctypes.c_size_t(0)
    assert lib.vdamp_plan_describe(None, None, 0, ctypes.byref(need)) == 1
    assert lib.vdamp_last_error()


def _ortho_status(taps, flags=0, ny=64, nx=64, levels=3, null_filter=False):
    lib = V.load_library()
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    a_ny = (ctypes.c_int32 * 1)(ny)
    a_nx = (ctypes.c_int32 * 1)(nx)
    a_h = None if null_filter else (ctypes.c_double * max(len(taps), 1))(*taps)
    st = lib.vdamp_plan_ortho(ctypes.byref(h), 1, a_ny, a_nx, levels, a_h, len(taps), flags,
                              ctypes.byref(wsb))
    return st, lib.vdamp_last_error().decode()


def test_plan_ortho_rejects_bad_filters_before_any_launch():
    """vdamp_plan_ortho checks the filter on the host: null, odd or out-of-range
    length, non-finite taps and a filter that is not orthonormal are argument errors;
    the Haar-pass tuner is not offered; shapes follow vdamp_plan's rules."""
    from paper_1911_01234_amd import filters
    db2 = list(filters.daubechies(2))
    assert _ortho_status(db2, null_filter=True)[0] == 1
    assert _ortho_status(db2[:3])[0] == 1                       # odd length
    assert _ortho_status([])[0] == 1                            # empty
    assert _ortho_status([0.0] * 66)[0] == 1                    # longer than 64
    assert _ortho_status([1.0, 1.0])[0] == 1                    # sum h = 2, not sqrt 2
    assert _ortho_status([0.5, 0.5, 0.5, 0.5])[0] == 1          # not orthogonal to its shifts
    assert _ortho_status([float("nan"), 1.0])[0] == 1
    assert _ortho_status(db2, flags=V.VDAMP_FLAG_AUTOTUNE)[0] == 3
    assert _ortho_status(db2, ny=60)[0] == 2
    st, msg = _ortho_status(db2, levels=0)
    assert st == 3 and msg


def test_group_pairs_refused_outside_2d_haar_plans():
    """VDAMP_FLAG_GROUP_PAIRS (joint thresholding of horizontal pairs) is a 2D Haar
    option: general-wavelet and volume plans refuse it on the host, before anything is
    allocated; an unknown flag bit above it stays an argument error."""
    from paper_1911_01234_amd import filters
    st, msg = _ortho_status(list(filters.daubechies(2)), flags=V.VDAMP_FLAG_GROUP_PAIRS)
    assert st == 3 and "GROUP_PAIRS" in msg
    lib = V.load_library()
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    one = lambda v: (ctypes.c_int32 * 1)(v)
    st = lib.vdamp_plan_3d(ctypes.byref(h), 1, one(32), one(32), one(32), 2, V.VDAMP_FLAG_GROUP_PAIRS,
                           ctypes.byref(wsb))
    assert st == 3 and "GROUP_PAIRS" in lib.vdamp_last_error().decode()
    st = lib.vdamp_plan(ctypes.byref(h), 1, one(64), one(64), 3, 0, 1 << 9, ctypes.byref(wsb))
    assert st == 1
