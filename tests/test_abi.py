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
    assert lib.sgrid_set_sweep_config(8, 1) == E_INVALID
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


def test_new_symbols_reject_invalid_arguments(lib):
    P = ctypes.c_void_p
    lib.sgrid_mlp_apply_gradient.argtypes = [P, P, ctypes.c_float, P]
    assert lib.sgrid_mlp_apply_gradient(None, P(16), 1e-3, None) == E_INVALID
    assert lib.sgrid_mlp_apply_gradient(P(64), None, 1e-3, None) == E_INVALID
    assert lib.sgrid_mlp_apply_gradient(P(64), P(16), -1.0, None) == E_INVALID
    f = lib.sgrid_compute_near_surface_integrals_factorised
    f.argtypes = [P, P, P, P, P]
    assert f(None, P(16), P(32), P(48), None) == E_INVALID
    assert f(P(64), None, P(32), P(48), None) == E_INVALID
    assert f(P(64), P(16), None, P(48), None) == E_INVALID
    assert f(P(64), P(16), P(16), P(48), None) == E_INVALID    # phi and vfrac aliased
    assert f(P(64), P(16), P(32), P(32), None) == E_INVALID    # vfrac and out aliased
    assert f(P(64), P(16), P(36), P(48), None) == E_INVALID    # misaligned
    # the particle sort: checks before any use of the grid
    ws = lib.sgrid_sort_particles_workspace_size
    ws.argtypes = [P, ctypes.c_int64, P]
    nb = ctypes.c_int64(-1)
    assert ws(None, 10, ctypes.byref(nb)) == E_INVALID
    assert ws(P(64), 10, None) == E_INVALID
    assert ws(P(64), -1, ctypes.byref(nb)) == E_INVALID
    assert ws(P(64), 1 << 32, ctypes.byref(nb)) == E_INVALID
    srt = lib.sgrid_sort_particles
    srt.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P]
    assert srt(None, P(16), 4, P(32), P(48), P(64), 1 << 20, None) == E_INVALID
    assert srt(P(64), P(16), -1, P(32), P(48), P(64), 1 << 20, None) == E_INVALID
    assert srt(P(64), None, 4, P(32), P(48), P(64), 1 << 20, None) == E_INVALID
    assert srt(P(64), P(16), 4, P(32), P(48), None, 1 << 20, None) == E_INVALID   # no workspace
    assert srt(P(64), P(16), 4, P(16), P(48), P(64), 1 << 20, None) == E_INVALID  # pos aliased
    assert srt(P(64), P(18), 4, P(32), P(48), P(64), 1 << 20, None) == E_INVALID  # misaligned
    # the allocation-free learned integrals: checks before any use of the grid
    na = lib.sgrid_compute_near_surface_integrals_noalloc
    na.argtypes = [P, P, P, P, P, P]
    assert na(None, P(16), P(64), P(32), None, None) == E_INVALID
    assert na(P(64), P(16), None, P(32), None, None) == E_INVALID                # no model
    assert na(P(64), None, P(64), P(32), None, None) == E_INVALID
    assert na(P(64), P(20), P(64), P(32), None, None) == E_INVALID               # misaligned


def _fake(cls, **attrs):
    """An object of a binding class whose handle is never used: the binding's
    own argument checks must reject the call before reaching the library."""
    obj = cls.__new__(cls)
    obj._h = ctypes.c_void_p(1)
    for k, v in attrs.items():
        setattr(obj, k, v)
    return obj


def test_binding_rejects_wrong_dtypes_and_sizes():
    torch = pytest.importorskip("torch")
    import paper_2512_11473_amd as sg
    f32, bf16, f64, i64 = torch.float32, torch.bfloat16, torch.float64, torch.int64
    m = _fake(sg.Mlp)
    B = 8
    x, y = torch.zeros(B, 216), torch.zeros(B, 4)
    bad = [
        lambda: m.forward(x, torch.zeros(B, 4, dtype=bf16)),              # y of half the bytes
        lambda: m.forward(x.to(f64), y),
        lambda: m.backward(x.to(bf16), y, torch.zeros(sg.MLP_N_PARAMS)),
        lambda: m.backward(x, y.to(f64), torch.zeros(sg.MLP_N_PARAMS)),
        lambda: m.backward(x, y, torch.zeros(sg.MLP_N_PARAMS, dtype=f64)),
        lambda: m.backward(x, y, torch.zeros(sg.MLP_N_PARAMS - 1)),
        lambda: m.train_step(x.to(f64), y, [1, 1, 1, 1], 1e-3),
        lambda: m.train_step(x, y.to(bf16), [1, 1, 1, 1], 1e-3),
        lambda: m.train_step(x, y, [1, 1, 1], 1e-3),                     # C reads 4 weights
        lambda: m.train_step(x, y, [1, 1, 1, 1, 1], 1e-3),
        lambda: m.train_step(x, y, [1, 1, 1, 1], 1e-3, torch.zeros(2)),   # loss is one float
        lambda: m.train_step(x, y, [1, 1, 1, 1], 1e-3, torch.zeros(1, dtype=f64)),
        lambda: m.apply_gradient(torch.zeros(sg.MLP_N_PARAMS, dtype=f64), 1e-3),
        lambda: m.apply_gradient(torch.zeros(10), 1e-3),
    ]
    g = _fake(sg.Grid, n_coarse=4, h=1 / 16, n_packages=10, n_core=3)
    nt = g.n_total
    bad += [
        lambda: sg.gather_windows(g, torch.zeros(nt, 64, dtype=f64)),
        lambda: sg.gather_windows(g, torch.zeros(nt - 1, 64)),
        lambda: sg.compute_near_surface_integrals(g, torch.zeros(nt, 64), torch.zeros(4, 3 * 64),
                                                  n_fallback=torch.zeros(1, dtype=i64)),
        lambda: sg.compute_near_surface_integrals(g, torch.zeros(nt, 64), torch.zeros(4, 3 * 64),
                                                  n_fallback=torch.zeros(0, dtype=torch.int32)),
        lambda: sg.compute_near_surface_integrals(g, torch.zeros(nt, 64), torch.zeros(4, 3 * 64), model=object()),
        lambda: sg.compute_near_surface_integrals_factorised(g, torch.zeros(nt, 64), torch.zeros(nt - 1, 64),
                                                             torch.zeros(4, 3 * 64)),
        lambda: sg.compute_near_surface_integrals_factorised(g, torch.zeros(nt, 64), torch.zeros(nt, 64, dtype=f64),
                                                             torch.zeros(4, 3 * 64)),
        lambda: sg.compute_near_surface_integrals_factorised(g, torch.zeros(nt, 64), torch.zeros(nt, 64),
                                                             torch.zeros(4, 2 * 64)),
    ]
    b = _fake(sg.Batch, n_total=20)
    bad += [
        lambda: b.autotune(torch.zeros(20, 64), torch.zeros(19, 64)),
        lambda: b.autotune(torch.zeros(20, 64, dtype=f64), torch.zeros(20, 64)),
        lambda: b.autotune(torch.zeros(21, 64), torch.zeros(20, 64)),
        lambda: b.reinitialize(torch.zeros(20, 64), torch.zeros(20, 64, dtype=f64), 1),
        lambda: b.reinitialize(torch.zeros(20, 64), torch.zeros(19, 64), 1),
    ]
    try:
        for call in bad:
            with pytest.raises((TypeError, ValueError)) as e:
                call()
            # the dtype / size check fired, not the later device-tensor check
            assert "device tensor" not in str(e.value), str(e.value)
        # control: well-formed host tensors get past those checks to that one
        with pytest.raises(ValueError, match="device tensor"):
            m.train_step(x, y, [1, 1, 1, 1], 1e-3, torch.zeros(1))
    finally:
        for obj in (m, g, b):   # the fake handles must never reach destroy
            obj._h = None
