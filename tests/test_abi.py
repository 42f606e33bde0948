"""C-ABI checks that need no GPU: the library loads, exports every function
include/lf2.h declares, and rejects bad arguments before any HIP call."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lf2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf2_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1508_05610_amd import _lib
    return _lib


def test_exports_every_declared_symbol(lib):
    so = lib.load()
    names = header_functions()
    assert "lf2_fft_plan" in names and "lf2_poisson_solve" in names
    for n in names:
        assert hasattr(so, n), f"{n} declared in lf2.h but not exported"
    # the binding covers the same names
    assert set(names) <= set(lib.exported_names())


def test_version_and_status_strings(lib):
    assert "gfx950" in lib.lf2_version()
    assert lib.status_string(-2) == "LF2_ERR_UNSUPPORTED"
    assert lib.status_string(0) == "LF2_OK"


@pytest.mark.parametrize("sizes,halo,ncomp,kind,dim,expect", [
    ((32, 32, 32), 0, 1, 0, 2, -2),          # 2-d lattices have no FFT
    ((32, 32, 32), -1, 1, 0, 3, -1),         # negative halo
    ((32, 32, 32), 0, 0, 0, 3, -1),          # ncomp < 1
    ((0, 32, 32), 0, 1, 0, 3, -1),           # empty extent
    ((33, 32, 32), 0, 1, 1, 3, -2),          # prime factor 11
    ((14, 32, 32), 0, 1, 0, 3, -2),          # prime factor 7
    ((31, 32, 32), 0, 1, 0, 3, -2),          # odd N0 for r2c
    ((32, 32, 32), 0, 1, 7, 3, -1),          # bad kind
    ((16384, 32, 32), 0, 1, 1, 3, -2),       # line longer than the run-time kernels take
    ((32, 3 * 8192, 32), 0, 1, 1, 3, -2),    # likewise along y
    ((7 * 16, 32, 32), 0, 1, 1, 3, -2),      # prime factor 7 with a power of two
])
def test_plan_validation(lib, sizes, halo, ncomp, kind, dim, expect):
    st = lib.lf2_fft_plan_status(sizes, halo, ncomp, kind, dim=dim)
    assert st == expect, (st, lib.last_error())
    assert lib.last_error()


@pytest.mark.parametrize("sizes,ncomp,kind", [
    ((15, 32, 32), 1, 1),          # both 3 and 5 in one extent
    ((15 * 16, 9 * 128, 45), 1, 1),
    ((18, 25, 27), 1, 0),          # r2c with N0/2 = 9
    ((144, 360, 450), 1, 0),
    ((720, 900, 8), 3, 1),
    ((32, 32, 32), 4, 0),          # four components: run-time kernels along x
])
def test_plan_accepts_any_235_extent(lib, sizes, ncomp, kind):
    """Every 2^a 3^b 5^c extent passes validation: without a GPU the call then
    fails only at the device query (LF2_ERR_DEVICE), never as unsupported."""
    st = lib.lf2_fft_plan_status(sizes, 0, ncomp, kind)
    assert st in (lib.LF2_OK, lib.LF2_ERR_DEVICE), (st, lib.last_error())


def test_null_plan_calls(lib):
    so = lib.load()
    assert so.lf2_fft_execute(None, -1, None, None, None) == lib.LF2_ERR_INVALID_ARG
    assert so.lf2_poisson_solve(None, None, None, 1.0, 0, 0, None, None, None, None, None) == -1
    assert so.lf2_power_spectrum(None, None, 0, 8, 1.0, None, None, None, None) == -1
    assert so.lf2_plan_destroy(None) == -1
    assert so.lf2_fft_plan(None, None, 1, 0, 0) == -1


def test_python_binding_raises(lib):
    with pytest.raises(lib.LF2Error) as ei:
        lib.lf2_fft_plan((7, 8, 8), 0, 1, 0)
    assert ei.value.status == lib.LF2_ERR_UNSUPPORTED


def test_variant_calls_validate(lib):
    so = lib.load()
    import ctypes
    v = ctypes.c_int32()
    assert so.lf2_plan_get_tuning(None, 1, ctypes.byref(v), None, None, None) == lib.LF2_ERR_INVALID_ARG
    assert so.lf2_plan_set_tuning(None, 2, 1, 16) == lib.LF2_ERR_INVALID_ARG


def test_unknown_plan_flag(lib):
    st = lib.lf2_fft_plan_status((32, 32, 32), 0, 1, 0, flags=0x20)
    assert st == lib.LF2_ERR_UNSUPPORTED


def test_layout_flag_validation(lib):
    # in place needs halo 0
    assert lib.lf2_fft_plan_status((32, 32, 32), 1, 1, 0, flags=lib.LF2_IN_PLACE) == \
        lib.LF2_ERR_UNSUPPORTED
    assert lib.lf2_fft_plan_status((32, 32, 32), 1, 1, 1, flags=lib.LF2_IN_PLACE) == \
        lib.LF2_ERR_UNSUPPORTED


def test_field_ops_validate(lib):
    import ctypes
    so = lib.load()
    lat = lib.lf2_lattice(3, 1, (ctypes.c_int64 * 3)(8, 8, 8))
    assert so.lf2_update_halo(ctypes.byref(lat), 1, 4, None, None) == lib.LF2_ERR_INVALID_ARG
    assert so.lf2_update_halo(ctypes.byref(lat), 1, 2, 256, None) == lib.LF2_ERR_UNSUPPORTED
    assert so.lf2_update_halo(None, 1, 4, 256, None) == lib.LF2_ERR_INVALID_ARG
    assert so.lf2_gradient(ctypes.byref(lat), 1, 256, 256, 1.0, None) == lib.LF2_ERR_INVALID_ARG
    assert so.lf2_gradient(ctypes.byref(lat), 1, 256, 512, 0.0, None) == lib.LF2_ERR_INVALID_ARG
    lat0 = lib.lf2_lattice(3, 0, (ctypes.c_int64 * 3)(8, 8, 8))
    assert so.lf2_gradient(ctypes.byref(lat0), 1, 256, 512, 1.0, None) == lib.LF2_ERR_INVALID_ARG
    wide = lib.lf2_lattice(3, 9, (ctypes.c_int64 * 3)(8, 8, 8))
    assert so.lf2_update_halo(ctypes.byref(wide), 1, 4, 256, None) == lib.LF2_ERR_UNSUPPORTED
