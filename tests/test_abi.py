"""The C ABI library loads, exports every symbol include/sgrid.h declares, and
rejects invalid arguments with SGRID_E_INVALID before touching the device
(runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgrid.h")
LIB = os.path.join(ROOT, "paper_2512_11473_amd", "libsgrid.so")
E_INVALID = 1


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgrid_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2512_11473_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n


def test_invalid_arguments_rejected_without_device(lib):
    P = ctypes.c_void_p
    lib.sgrid_last_error.restype = ctypes.c_char_p
    lib.sgrid_build_packages.argtypes = [P, P, P, P]
    out = ctypes.c_void_p(123)
    assert lib.sgrid_build_packages(None, None, None, ctypes.byref(out)) == E_INVALID
    assert out.value is None
    assert b"NULL" in lib.sgrid_last_error()

    class Desc(ctypes.Structure):
        _fields_ = [("n_coarse", ctypes.c_int32), ("h", ctypes.c_double)]

    d = Desc(0, 0.1)
    assert lib.sgrid_build_packages(ctypes.byref(d), P(16), None, ctypes.byref(out)) == E_INVALID
    d = Desc(8, -1.0)
    assert lib.sgrid_build_packages(ctypes.byref(d), P(16), None, ctypes.byref(out)) == E_INVALID
    d = Desc(4000, 0.1)   # 6.4e10 cells: beyond 32-bit package ids
    assert lib.sgrid_build_packages(ctypes.byref(d), P(16), None, ctypes.byref(out)) == 4
    lib.sgrid_reinitialize.argtypes = [P, ctypes.c_int, P, P, ctypes.c_int32, P]
    assert lib.sgrid_reinitialize(None, 0, P(16), P(32), 1, None) == E_INVALID
    lib.sgrid_compute_gradient.argtypes = [P, ctypes.c_int, P, P, P]
    assert lib.sgrid_compute_gradient(None, 0, P(16), P(32), None) == E_INVALID
    lib.sgrid_probe_particles.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int64, P, P, P]
    assert lib.sgrid_probe_particles(None, 0, None, None, None, 0, None, None, None) == E_INVALID
    lib.sgrid_compute_near_surface_integrals.argtypes = [P, P, P, P, P, P]
    assert lib.sgrid_compute_near_surface_integrals(None, None, None, None, None, None) == E_INVALID
    lib.sgrid_set_sweep_config.argtypes = [ctypes.c_int32, ctypes.c_int32]
    assert lib.sgrid_set_sweep_config(7, 1) == E_INVALID
    assert lib.sgrid_set_sweep_config(0, 9) == E_INVALID
    lib.sgrid_sequential_update.argtypes = [P, ctypes.c_int, P, ctypes.c_double, P]
    assert lib.sgrid_sequential_update(None, 0, P(16), 1e-3, None) == E_INVALID
    lib.sgrid_compute_laplacian.argtypes = [P, ctypes.c_int, P, P, P]
    assert lib.sgrid_compute_laplacian(None, 0, P(16), P(32), None) == E_INVALID
    assert lib.sgrid_compute_laplacian(P(64), 0, P(16), P(16), None) == E_INVALID
    lib.sgrid_autotune_sweep.argtypes = [P, ctypes.c_int, P, P, ctypes.c_int32, P, P, P, P]
    assert lib.sgrid_autotune_sweep(None, 0, P(16), P(32), 1, None, None, None, None) == E_INVALID
    assert lib.sgrid_autotune_sweep(P(64), 0, P(16), P(32), 0, None, None, None, None) == E_INVALID
    # the multi-resolution layer, the sign correction and the integral field
    lib.sgrid_build_packages_refined.argtypes = [P, P, P, P]
    assert lib.sgrid_build_packages_refined(None, P(16), None, ctypes.byref(out)) == E_INVALID
    assert lib.sgrid_build_packages_refined(P(64), P(16), None, None) == E_INVALID
    lib.sgrid_correct_signs.argtypes = [P, P, P, P, P]
    assert lib.sgrid_correct_signs(None, P(16), P(16), None, None) == E_INVALID
    d = Desc(8, 0.1)
    assert lib.sgrid_correct_signs(ctypes.byref(d), None, P(16), None, None) == E_INVALID
    assert lib.sgrid_correct_signs(ctypes.byref(d), P(18), P(16), None, None) == E_INVALID   # misaligned
    d = Desc(5000, 0.1)
    assert lib.sgrid_correct_signs(ctypes.byref(d), P(16), P(16), None, None) == E_INVALID
    d = Desc(8, 0.0)
    assert lib.sgrid_correct_signs(ctypes.byref(d), P(16), P(16), None, None) == E_INVALID
    lib.sgrid_correct_package_signs.argtypes = [P, ctypes.c_int, P, P, P]
    assert lib.sgrid_correct_package_signs(None, 0, P(16), None, None) == E_INVALID
    assert lib.sgrid_correct_package_signs(P(64), 0, None, None, None) == E_INVALID
    assert lib.sgrid_correct_package_signs(P(64), 7, P(16), None, None) == E_INVALID
    assert lib.sgrid_correct_package_signs(P(64), 1, P(20), None, None) == E_INVALID   # misaligned FP64
    lib.sgrid_compute_integral_field.argtypes = [P, P, P, P]
    assert lib.sgrid_compute_integral_field(None, P(16), P(32), None) == E_INVALID
    assert lib.sgrid_compute_integral_field(P(64), P(16), P(16), None) == E_INVALID   # aliased
    lib.sgrid_probe_integral_field.argtypes = [P, P, P, ctypes.c_int64, P, P]
    assert lib.sgrid_probe_integral_field(None, P(16), P(16), 1, P(16), None) == E_INVALID
    assert lib.sgrid_probe_integral_field(P(64), P(16), P(16), -1, P(16), None) == E_INVALID
    assert lib.sgrid_probe_integral_field(P(64), P(16), P(16), 0, P(16), None) == 0   # nothing to do
    lib.sgrid_destroy.argtypes = [P]
    assert lib.sgrid_destroy(None) == 0
    assert lib.sgrid_version() >= 10000
