"""The C ABI library loads, exports every declared entry point, and rejects
bad arguments on the host (no GPU needed for any of these calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1509_07691_amd import fslbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fslbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fslbm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fslbm.LIB_PATH):
        pytest.skip("libfslbm.so not built")
    return fslbm.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fslbm_create", "fslbm_set_params", "fslbm_step", "fslbm_read_fill",
                     "fslbm_read_pressure", "fslbm_read_curvature", "fslbm_read_velocity",
                     "fslbm_mass", "fslbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_python_binding_uses_the_c_names():
    for name in declared_functions():
        if name in ("fslbm_last_error",):
            continue
        assert hasattr(fslbm, name), name


def test_required_bytes_and_shape_errors(lib):
    b32 = fslbm.fslbm_required_bytes(32, 32, 32, fslbm.FSLBM_F32)
    b64 = fslbm.fslbm_required_bytes(32, 32, 32, fslbm.FSLBM_F64)
    b16 = fslbm.fslbm_required_bytes(32, 32, 32, fslbm.FSLBM_F16_STORE)
    n = 32 ** 3
    assert b16 < b32 < b64
    assert b32 >= 2 * 19 * 4 * n  # two distribution buffers
    with pytest.raises(fslbm.FslbmError) as e:
        fslbm.fslbm_required_bytes(2, 32, 32, fslbm.FSLBM_F32)
    assert e.value.code == -2
    with pytest.raises(fslbm.FslbmError) as e:
        fslbm.fslbm_required_bytes(2048, 2048, 1024, fslbm.FSLBM_F32)
    assert e.value.code == -2
    with pytest.raises(fslbm.FslbmError) as e:
        fslbm.fslbm_required_bytes(8, 8, 8, 7)
    assert e.value.code == -1


def test_pull_copy_sizes_and_argument_errors(lib):
    """The pull-copy measurement aid: 19 planes of the lattice's plane stride
    (N rounded up to 64, plus a 1024-element gap); every argument error is
    reported before any device call."""
    n = 13 * 17 * 19
    ns = (n + 63) // 64 * 64 + 1024
    for prec, s in ((fslbm.FSLBM_F64, 8), (fslbm.FSLBM_F32, 4), (fslbm.FSLBM_F16_STORE, 2), (fslbm.FSLBM_BF16_STORE, 2)):
        assert fslbm.fslbm_pull_copy_bytes(13, 17, 19, prec) == 19 * ns * s
    need = 19 * ns * 4
    cases = [((2, 17, 19, fslbm.FSLBM_F32, 1, 2, need, 0, 3), -2),   # extent below 3
             ((13, 17, 19, 9, 1, 2, need, 0, 3), -1),                 # precision
             ((13, 17, 19, fslbm.FSLBM_F32, 0, 2, need, 0, 3), -1),   # NULL source
             ((13, 17, 19, fslbm.FSLBM_F32, 1, 1, need, 0, 3), -1),   # src == dst
             ((13, 17, 19, fslbm.FSLBM_F32, 1, 2, need - 1, 0, 3), -2),  # buffers too small
             ((13, 17, 19, fslbm.FSLBM_F32, 1, 2, need, 0, 0), -1)]   # no launch
    for args, code in cases:
        with pytest.raises(fslbm.FslbmError) as e:
            fslbm.fslbm_pull_copy_time(*args)
        assert e.value.code == code, args


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    fill = np.zeros(8 * 8 * 8)
    h = ctypes.c_void_p()
    dp = fill.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # null workspace
    assert lib.fslbm_create(8, 8, 8, 1, 0, dp, None, None, 0, None, ctypes.byref(h)) == -1
    # misaligned workspace pointer
    assert lib.fslbm_create(8, 8, 8, 1, 0, dp, None, ctypes.c_void_p(16), 1 << 30, None, ctypes.byref(h)) == -1
    # workspace too small
    assert lib.fslbm_create(8, 8, 8, 1, 0, dp, None, ctypes.c_void_p(1 << 20), 64, None, ctypes.byref(h)) == -2
    # the FD model needs every extent >= 10; LSQR gets past that check
    f9 = np.zeros(9 * 32 * 32)
    d9 = f9.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.fslbm_create(9, 32, 32, 1, 0, d9, None, ctypes.c_void_p(1 << 20), 64, None, ctypes.byref(h)) == -2
    assert b"FD" in lib.fslbm_last_error()
    assert lib.fslbm_create(9, 32, 32, 1, 1, d9, None, ctypes.c_void_p(1 << 20), 64, None, ctypes.byref(h)) == -2
    assert b"workspace" in lib.fslbm_last_error()
    # unknown curvature model
    assert lib.fslbm_create(8, 8, 8, 1, 5, dp, None, ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h)) == -1
    assert b"curvature" in lib.fslbm_last_error()
    # null handle
    assert lib.fslbm_step(None, 1) == -4
    assert lib.fslbm_set_params(None, 0.0, 1.0, 1.0, 1.0) == -4


def _film_on_wall(thickness, n=16):
    """A liquid film of the given thickness (cells) on the wall z = 0 of an
    n^3 box, gas above (exact cell fractions)."""
    fill = np.zeros((n, n, n))
    obst = np.zeros((n, n, n), np.uint8)
    obst[0] = 1
    full = int(np.floor(thickness))
    fill[1:1 + full] = 1.0
    if thickness > full:
        fill[1 + full] = thickness - full
    return fill, obst


@pytest.mark.parametrize("thickness", [0.6, 1.0])
def test_create_rejects_films_thinner_than_one_cell(lib, thickness):
    """Sec. II.D, Fig. limitation: a liquid film on a wall must hold at least
    one liquid cell; thinner films are rejected on the host, before any
    device call (the workspace pointer here is never dereferenced)."""
    fill, obst = _film_on_wall(thickness)
    h = ctypes.c_void_p()
    rc = lib.fslbm_create(16, 16, 16, 1, 1, fill.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          obst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.c_void_p(1 << 20), 1 << 62,
                          None, ctypes.byref(h))
    assert rc == fslbm.FSLBM_E_TOPOLOGY
    assert b"thinner than one cell" in lib.fslbm_last_error()
    assert not h.value


def test_create_rejects_gas_layers_thinner_than_one_cell(lib):
    fill = np.ones((16, 16, 16))
    fill[5] = 0.3  # a gas layer of 0.7 cells between liquid
    h = ctypes.c_void_p()
    rc = lib.fslbm_create(16, 16, 16, 1, 1, fill.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None,
                          ctypes.c_void_p(1 << 20), 1 << 62, None, ctypes.byref(h))
    assert rc == fslbm.FSLBM_E_TOPOLOGY
