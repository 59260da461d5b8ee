"""sgrid: contiguous narrow-band sparse grids on MI355X.

Thin Python binding of the C ABI in ``include/sgrid.h`` (``libsgrid.so``).
It only marshals arguments: torch tensors supply device memory and the
current HIP stream, and every step of the hot path runs in the library's HIP
kernels.  There is no CPU fallback: importing the binding without a built
library, or calling it without a GPU, raises.

Names follow the C ABI without the ``sgrid_`` prefix.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

__all__ = [
    "SgridError", "Grid", "load", "build_packages", "build_packages_refined", "correct_signs",
    "correct_package_signs", "fill_far_field",
    "reinitialize",
    "compute_gradient", "compute_gradient_packed", "probe_particles", "probe_particles_packed", "compute_near_surface_integrals", "set_sweep_config",
    "compute_integral_field", "probe_integral_field",
    "sequential_update", "compute_laplacian",
    "autotune_sweep", "SWEEP_TUNE_CANDIDATES",
    "Mlp", "gather_windows", "MLP_N_PARAMS", "Batch", "compute_near_surface_integrals_noalloc",
    "sort_particles", "sort_workspace_bytes",
    "LIB_PATH", "FAR_FIELD_IN_H",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsgrid.so")
FAR_FIELD_IN_H = 16.0
_lib = None
_P = ctypes.c_void_p


class SgridError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"sgrid status {status}: {message}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("n_coarse", ctypes.c_int32), ("h", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("n_coarse", ctypes.c_int32), ("h", ctypes.c_double), ("n_packages", ctypes.c_int64),
                ("n_core", ctypes.c_int64), ("cell_pkg", _P), ("pkg_cell", _P), ("pkg_type", _P),
                ("pkg_nbr", _P), ("core_list", _P), ("sweep_order", _P), ("rank_map", _P),
                ("rank_row", ctypes.c_int32)]


_SIGNATURES = {
    "sgrid_last_error": (ctypes.c_char_p, []),
    "sgrid_version": (ctypes.c_int32, []),
    "sgrid_build_packages": (ctypes.c_int, [ctypes.POINTER(_Desc), _P, _P, ctypes.POINTER(_P)]),
    "sgrid_build_packages_refined": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_P)]),
    "sgrid_correct_signs": (ctypes.c_int, [ctypes.POINTER(_Desc), _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "sgrid_correct_package_signs": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "sgrid_get_info": (ctypes.c_int, [_P, ctypes.POINTER(_Info)]),
    "sgrid_destroy": (ctypes.c_int, [_P]),
    "sgrid_fill_far_field": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sgrid_reinitialize": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int32, _P]),
    "sgrid_compute_gradient": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "sgrid_compute_gradient_packed": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "sgrid_probe_particles_packed": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int64, _P, _P, _P]),
    "sgrid_probe_particles": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_int64, _P, _P, _P]),
    "sgrid_compute_near_surface_integrals": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "sgrid_compute_near_surface_integrals_factorised": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sgrid_compute_integral_field": (ctypes.c_int, [_P, _P, _P, _P]),
    "sgrid_probe_integral_field": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P]),
    "sgrid_set_sweep_config": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "sgrid_sequential_update": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_double, _P]),
    "sgrid_compute_laplacian": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "sgrid_autotune_sweep": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int32, _P,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _P]),
    "sgrid_mlp_create": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "sgrid_mlp_destroy": (ctypes.c_int, [_P]),
    "sgrid_mlp_get_params": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "sgrid_mlp_set_state": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64]),
    "sgrid_mlp_set_gate": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "sgrid_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "sgrid_mlp_backward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P]),
    "sgrid_mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_float, _P, _P]),
    "sgrid_mlp_apply_gradient": (ctypes.c_int, [_P, _P, ctypes.c_float, _P]),
    "sgrid_gather_windows": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sgrid_compute_near_surface_integrals_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "sgrid_sort_particles_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "sgrid_sort_particles": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_int64, _P]),
    "sgrid_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "sgrid_batch_destroy": (ctypes.c_int, [_P]),
    "sgrid_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), _P]),
    "sgrid_batch_set_config": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "sgrid_batch_autotune": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32), _P]),
    "sgrid_batch_reinitialize": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
}


def load():
    """Load libsgrid.so (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        # the HIP runtime must be the one torch already loaded
        torch.cuda.is_available()
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        msg = load().sgrid_last_error()
        raise SgridError(status, msg.decode() if msg else "")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return 0
    if t.dtype == torch.float64:
        return 1
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, name: str, numel: int):
    """t must be a float32 tensor of exactly `numel` elements (the library
    cannot check either)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} values (got {t.numel()})")


def _counter(t, name: str):
    """A device counter the library writes one 32-bit unsigned value to."""
    if t.dtype not in (torch.int32, torch.uint32) or t.numel() < 1:
        raise TypeError(f"{name} must be an int32 or uint32 tensor of at least one element")
    return _dev(t, name)


def _hip_runtime():
    """The HIP runtime this process already loaded (torch's), found by path."""
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1] if len(line.split()) >= 6 else ""
            if os.path.basename(path).startswith("libamdhip64.so"):
                return ctypes.CDLL(path)
    raise SgridError(3, "the HIP runtime is not loaded in this process")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Grid:
    """An activated narrow band: owns the library's index tables."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        info = _Info()
        _check(load().sgrid_get_info(self._h, ctypes.byref(info)))
        self.n_coarse = int(info.n_coarse)
        self.h = float(info.h)
        self.n_packages = int(info.n_packages)
        self.n_core = int(info.n_core)
        self._info = info

    @property
    def handle(self):
        if self._h is None:
            raise SgridError(5, "grid already destroyed")
        return self._h

    @property
    def n_total(self) -> int:
        return self.n_packages + 2

    @property
    def far_field(self) -> float:
        return FAR_FIELD_IN_H * self.h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _check(load().sgrid_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def tables(self) -> dict:
        """Copies of the index tables as device tensors (for checks)."""
        hip = _hip_runtime()
        hip.hipMemcpy.argtypes = [_P, _P, ctypes.c_size_t, ctypes.c_int]
        hip.hipMemcpy.restype = ctypes.c_int
        info = self._info
        M, nt = self.n_coarse, self.n_total

        def grab(ptr, n, dtype, esize):
            t = torch.empty(n, dtype=dtype, device="cuda")
            if n:
                torch.cuda.synchronize()
                rc = hip.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(ptr), n * esize, 3)
                if rc != 0:
                    raise SgridError(3, f"hipMemcpy failed ({rc})")
            return t

        return {
            "cell_pkg": grab(info.cell_pkg, M ** 3, torch.int32, 4),
            "pkg_cell": grab(info.pkg_cell, nt, torch.int32, 4),
            "pkg_type": grab(info.pkg_type, nt, torch.uint8, 1),
            "pkg_nbr": grab(info.pkg_nbr, nt * 27, torch.int32, 4).view(nt, 27),
            "core_list": grab(info.core_list, self.n_core, torch.int32, 4),
            "sweep_order": grab(info.sweep_order, self.n_packages, torch.int32, 4),
            "rank_map": grab(info.rank_map, M * M * info.rank_row * 4, torch.int32, 4).view(M * M, info.rank_row, 4),
        }

    def empty_field(self, dtype=torch.float32, components: int = 1) -> torch.Tensor:
        shape = (self.n_total, 64) if components == 1 else (components, self.n_total, 64)
        return torch.empty(shape, dtype=dtype, device="cuda")


def build_packages(coarse_sdf: torch.Tensor, h: float, stream=None) -> Grid:
    """Activation, numbering and neighbour tables from the coarse distances
    (float32, M^3 values, x fastest)."""
    n = coarse_sdf.numel()
    M = int(round(n ** (1.0 / 3.0)))
    if M ** 3 != n:
        raise ValueError(f"coarse_sdf has {n} values, not a cube")
    if coarse_sdf.dtype != torch.float32:
        raise TypeError("coarse_sdf must be float32")
    desc = _Desc(M, float(h))
    out = ctypes.c_void_p()
    _check(load().sgrid_build_packages(ctypes.byref(desc), _dev(coarse_sdf, "coarse_sdf"), _stream(stream),
                                       ctypes.byref(out)))
    return Grid(out)


def build_packages_refined(coarse: Grid, child_sdf: Optional[torch.Tensor], stream=None) -> Grid:
    """The layer of doubled resolution built from `coarse`: child_sdf holds
    the distances at the eight children of each core cell of `coarse`
    (float32 [n_core, 8], core_list order, child bx + 2 by + 4 bz)."""
    if coarse.n_core > 0:
        if child_sdf is None or child_sdf.dtype != torch.float32 or child_sdf.numel() != 8 * coarse.n_core:
            raise ValueError(f"child_sdf must be float32 [{coarse.n_core}, 8]")
        ptr = _dev(child_sdf, "child_sdf")
    else:
        ptr = None
    out = ctypes.c_void_p()
    _check(load().sgrid_build_packages_refined(coarse.handle, ptr, _stream(stream), ctypes.byref(out)))
    return Grid(out)


def correct_signs(coarse_sdf: torch.Tensor, h: float, out: Optional[torch.Tensor] = None, stream=None) -> int:
    """Sign correction of coarse distances (float32, M^3 values) by diffusion
    from the core cells; writes `out` (default: in place) and returns the
    number of rounds that decided a cell."""
    n = coarse_sdf.numel()
    M = int(round(n ** (1.0 / 3.0)))
    if M ** 3 != n:
        raise ValueError(f"coarse_sdf has {n} values, not a cube")
    if coarse_sdf.dtype != torch.float32 or (out is not None and (out.dtype != torch.float32 or out.numel() != n)):
        raise TypeError("coarse_sdf and out must be float32 of the same size")
    out = coarse_sdf if out is None else out
    desc = _Desc(M, float(h))
    rounds = ctypes.c_int32()
    _check(load().sgrid_correct_signs(ctypes.byref(desc), _dev(coarse_sdf, "coarse_sdf"), _dev(out, "out"),
                                      _stream(stream), ctypes.byref(rounds)))
    return int(rounds.value)


def correct_package_signs(grid: Grid, phi: torch.Tensor, stream=None) -> int:
    """Sign correction of the inner packages' points of phi [P+2, 64] in place,
    by diffusion from the core packages and the far field; returns the number
    of rounds that decided a point."""
    if phi.numel() != grid.n_total * 64:
        raise ValueError("phi must be [P+2, 64]")
    rounds = ctypes.c_int32()
    _check(load().sgrid_correct_package_signs(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _stream(stream),
                                              ctypes.byref(rounds)))
    return int(rounds.value)


def fill_far_field(grid: Grid, phi: torch.Tensor, stream=None):
    _check(load().sgrid_fill_far_field(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _stream(stream)))


def reinitialize(grid: Grid, phi: torch.Tensor, scratch: torch.Tensor, n_iter: int, stream=None):
    if scratch.dtype != phi.dtype or scratch.numel() != phi.numel() or phi.numel() != grid.n_total * 64:
        raise ValueError("phi and scratch must both be [P+2, 64] of one dtype")
    _check(load().sgrid_reinitialize(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _dev(scratch, "scratch"),
                                     int(n_iter), _stream(stream)))


def sequential_update(grid: Grid, phi: torch.Tensor, delta: float, stream=None):
    """phi += delta at every point of every activated package."""
    if phi.numel() != grid.n_total * 64:
        raise ValueError("phi must be [P+2, 64]")
    _check(load().sgrid_sequential_update(grid.handle, _dtype_code(phi), _dev(phi, "phi"), float(delta),
                                          _stream(stream)))


def compute_laplacian(grid: Grid, phi: torch.Tensor, out: torch.Tensor, stream=None):
    """Seven-point Laplacian of phi at every point of every activated package."""
    if out.dtype != phi.dtype or out.numel() != phi.numel() or phi.numel() != grid.n_total * 64:
        raise ValueError("phi and out must both be [P+2, 64] of one dtype")
    _check(load().sgrid_compute_laplacian(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _dev(out, "out"),
                                          _stream(stream)))


def compute_gradient(grid: Grid, phi: torch.Tensor, grad: torch.Tensor, stream=None):
    if grad.dtype != phi.dtype or grad.numel() != 3 * phi.numel() or phi.numel() != grid.n_total * 64:
        raise ValueError("grad must be [3, P+2, 64] of phi's dtype")
    _check(load().sgrid_compute_gradient(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _dev(grad, "grad"),
                                         _stream(stream)))


def compute_gradient_packed(grid: Grid, phi: torch.Tensor, packed: torch.Tensor, stream=None):
    """(phi, gx, gy, gz) quadruples [P+2, 64, 4] for the packed probe."""
    if packed.dtype != phi.dtype or packed.numel() != 4 * phi.numel() or phi.numel() != grid.n_total * 64:
        raise ValueError("packed must be [P+2, 64, 4] of phi's dtype")
    _check(load().sgrid_compute_gradient_packed(grid.handle, _dtype_code(phi), _dev(phi, "phi"),
                                                _dev(packed, "packed"), _stream(stream)))


def probe_particles_packed(grid: Grid, packed: torch.Tensor, pos: torch.Tensor, phi_out: torch.Tensor,
                           normal_out: torch.Tensor, stream=None):
    n = pos.numel() // 3
    if pos.numel() != 3 * n or phi_out.numel() != n or normal_out.numel() != 3 * n:
        raise ValueError("pos [n,3], phi_out [n], normal_out [n,3] expected")
    for t in (pos, phi_out, normal_out):
        if t.dtype != packed.dtype:
            raise TypeError("all probe arrays must share the field's dtype")
    if packed.numel() != grid.n_total * 256:
        raise ValueError("packed must be [P+2, 64, 4]")
    _check(load().sgrid_probe_particles_packed(grid.handle, _dtype_code(packed), _dev(packed, "packed"),
                                               _dev(pos, "pos"), n, _dev(phi_out, "phi_out"),
                                               _dev(normal_out, "normal_out"), _stream(stream)))


def sort_workspace_bytes(grid: Grid, n: int) -> int:
    out = ctypes.c_int64()
    _check(load().sgrid_sort_particles_workspace_size(grid.handle, int(n), ctypes.byref(out)))
    return int(out.value)


def sort_particles(grid: Grid, pos: torch.Tensor, pos_sorted: torch.Tensor, perm: torch.Tensor,
                   workspace: Optional[torch.Tensor] = None, stream=None):
    """Counting sort of the particles by home package (Morton worklist order):
    pos_sorted[i] = pos[perm[i]].  `workspace` is a device tensor of at least
    sort_workspace_bytes(grid, n) bytes (allocated here when None)."""
    n = pos.numel() // 3
    _f32(pos, "pos", 3 * n)
    _f32(pos_sorted, "pos_sorted", 3 * n)
    if perm.dtype not in (torch.int32, torch.uint32) or perm.numel() != n:
        raise TypeError("perm must be an int32 or uint32 tensor of n elements")
    need = sort_workspace_bytes(grid, n)
    if workspace is None:
        workspace = torch.empty(max(need, 4), dtype=torch.uint8, device="cuda")
    have = workspace.numel() * workspace.element_size()
    if have < need:
        raise ValueError(f"workspace holds {have} bytes, the sort needs {need}")
    _check(load().sgrid_sort_particles(grid.handle, _dev(pos, "pos"), n, _dev(pos_sorted, "pos_sorted"),
                                       _dev(perm, "perm"), _dev(workspace, "workspace"), have, _stream(stream)))


def probe_particles(grid: Grid, phi: torch.Tensor, grad: torch.Tensor, pos: torch.Tensor,
                    phi_out: torch.Tensor, normal_out: torch.Tensor, stream=None):
    n = pos.numel() // 3
    if pos.numel() != 3 * n or phi_out.numel() != n or normal_out.numel() != 3 * n:
        raise ValueError("pos [n,3], phi_out [n], normal_out [n,3] expected")
    for t in (grad, pos, phi_out, normal_out):
        if t.dtype != phi.dtype:
            raise TypeError("all probe arrays must share phi's dtype")
    if phi.numel() != grid.n_total * 64 or grad.numel() != 3 * phi.numel():
        raise ValueError("phi [P+2, 64] and grad [3, P+2, 64] expected")
    _check(load().sgrid_probe_particles(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _dev(grad, "grad"),
                                        _dev(pos, "pos"), n, _dev(phi_out, "phi_out"),
                                        _dev(normal_out, "normal_out"), _stream(stream)))


def compute_near_surface_integrals(grid: Grid, phi: torch.Tensor, out: torch.Tensor, model=None,
                                   n_fallback: Optional[torch.Tensor] = None, stream=None):
    if phi.dtype != torch.float32 or out.dtype != torch.float32:
        raise TypeError("integrals are FP32")
    if out.numel() != 4 * grid.n_core * 64 or phi.numel() != grid.n_total * 64:
        raise ValueError("out must be [4, n_core*64]")
    nf = _counter(n_fallback, "n_fallback") if n_fallback is not None else None
    if model is not None and not isinstance(model, Mlp):
        raise TypeError("model must be an Mlp")
    mh = model.handle if model is not None else None
    _check(load().sgrid_compute_near_surface_integrals(grid.handle, _dev(phi, "phi"), mh, _dev(out, "out"), nf,
                                                       _stream(stream)))


def compute_near_surface_integrals_noalloc(grid: Grid, phi: torch.Tensor, out: torch.Tensor, model,
                                           n_fallback: Optional[torch.Tensor] = None, stream=None):
    """The learned integrals of compute_near_surface_integrals(model=...) with
    the fallback list in the library's fixed per-device array: no device
    allocation.  Calls that overlap on one GPU race."""
    if phi.dtype != torch.float32 or out.dtype != torch.float32:
        raise TypeError("integrals are FP32")
    if out.numel() != 4 * grid.n_core * 64 or phi.numel() != grid.n_total * 64:
        raise ValueError("out must be [4, n_core*64]")
    if not isinstance(model, Mlp):
        raise TypeError("model must be an Mlp")
    nf = _counter(n_fallback, "n_fallback") if n_fallback is not None else None
    _check(load().sgrid_compute_near_surface_integrals_noalloc(grid.handle, _dev(phi, "phi"), model.handle,
                                                               _dev(out, "out"), nf, _stream(stream)))


def compute_near_surface_integrals_factorised(grid: Grid, phi: torch.Tensor, vfrac: torch.Tensor,
                                              out: torch.Tensor, stream=None):
    """The plain integrals in two passes: cut fractions at every point into
    `vfrac` ([P+2, 64] FP32 workspace), then the 32 taps per core point."""
    for name, t in (("phi", phi), ("vfrac", vfrac), ("out", out)):
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
    if phi.numel() != grid.n_total * 64 or vfrac.numel() != grid.n_total * 64:
        raise ValueError("phi and vfrac must be [P+2, 64]")
    if out.numel() != 4 * grid.n_core * 64:
        raise ValueError("out must be [4, n_core*64]")
    _check(load().sgrid_compute_near_surface_integrals_factorised(grid.handle, _dev(phi, "phi"), _dev(vfrac, "vfrac"),
                                                                  _dev(out, "out"), _stream(stream)))


def compute_integral_field(grid: Grid, phi: torch.Tensor, field: torch.Tensor, stream=None):
    """(K_W, h K_grad) at every point of every activated package, packed
    [P+2, 64, 4] like compute_gradient_packed; far-field rows hold the
    one-sided constants."""
    if phi.dtype != torch.float32 or field.dtype != torch.float32:
        raise TypeError("the integral field is FP32")
    if phi.numel() != grid.n_total * 64 or field.numel() != grid.n_total * 256:
        raise ValueError("phi [P+2, 64] and field [P+2, 64, 4] expected")
    _check(load().sgrid_compute_integral_field(grid.handle, _dev(phi, "phi"), _dev(field, "field"),
                                               _stream(stream)))


def probe_integral_field(grid: Grid, field: torch.Tensor, pos: torch.Tensor, out: torch.Tensor, stream=None):
    """Trilinear interpolation of the integral field at particles: out [n, 4]."""
    n = pos.numel() // 3
    if pos.numel() != 3 * n or out.numel() != 4 * n:
        raise ValueError("pos [n,3] and out [n,4] expected")
    for t in (field, pos, out):
        if t.dtype != torch.float32:
            raise TypeError("the integral field probe is FP32")
    if field.numel() != grid.n_total * 256:
        raise ValueError("field must be [P+2, 64, 4]")
    _check(load().sgrid_probe_integral_field(grid.handle, _dev(field, "field"), _dev(pos, "pos"), n,
                                             _dev(out, "out"), _stream(stream)))


MLP_N_PARAMS = 44804


class Mlp:
    """Surrogate network handle (FP32 master parameters on the device)."""

    def __init__(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_N_PARAMS,):
            raise ValueError(f"expected {MLP_N_PARAMS} parameters")
        out = ctypes.c_void_p()
        _check(load().sgrid_mlp_create(p.ctypes.data_as(_P), ctypes.byref(out)))
        self._h = out

    @property
    def handle(self):
        if self._h is None:
            raise SgridError(5, "model already destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _check(load().sgrid_mlp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def state(self):
        """(params, adam_m, adam_v, step) as host arrays."""
        import numpy as np
        w, m, v = (np.empty(MLP_N_PARAMS, dtype=np.float32) for _ in range(3))
        step = ctypes.c_int64()
        _check(load().sgrid_mlp_get_params(self.handle, w.ctypes.data_as(_P), m.ctypes.data_as(_P),
                                           v.ctypes.data_as(_P), ctypes.byref(step)))
        return w, m, v, int(step.value)

    def set_state(self, adam_m, adam_v, step: int):
        import numpy as np
        m = np.ascontiguousarray(adam_m, dtype=np.float32)
        v = np.ascontiguousarray(adam_v, dtype=np.float32)
        _check(load().sgrid_mlp_set_state(self.handle, m.ctypes.data_as(_P), v.ctypes.data_as(_P), int(step)))

    def set_gate(self, tau: float, kw_lo: float = -0.05, kw_hi: float = 1.05):
        _check(load().sgrid_mlp_set_gate(self.handle, float(tau), float(kw_lo), float(kw_hi)))

    def forward(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        B = x.shape[0]
        if x.shape != (B, 216) or y.shape != (B, 4):
            raise ValueError("x [B,216] and y [B,4] float32 expected")
        _f32(x, "x", B * 216)
        _f32(y, "y", B * 4)
        _check(load().sgrid_mlp_forward(self.handle, _dev(x, "x"), B, _dev(y, "y"), _stream(stream)))

    def backward(self, x: torch.Tensor, dy: torch.Tensor, grad: torch.Tensor, stream=None):
        B = x.shape[0]
        if x.shape != (B, 216) or dy.shape != (B, 4):
            raise ValueError("x [B,216], dy [B,4], grad [44804] expected")
        _f32(x, "x", B * 216)
        _f32(dy, "dy", B * 4)
        _f32(grad, "grad", MLP_N_PARAMS)
        _check(load().sgrid_mlp_backward(self.handle, _dev(x, "x"), _dev(dy, "dy"), B, _dev(grad, "grad"),
                                         _stream(stream)))

    def _train_args(self, x, t, loss_weights, loss):
        import numpy as np
        B = x.shape[0]
        if x.shape != (B, 216) or t.shape != (B, 4):
            raise ValueError("x [B,216] and t [B,4] expected")
        _f32(x, "x", B * 216)
        _f32(t, "t", B * 4)
        lw = np.ascontiguousarray(loss_weights, dtype=np.float32)
        if lw.shape != (4,):
            raise ValueError("loss_weights must hold exactly 4 values")
        if loss is not None:
            _f32(loss, "loss", 1)
        lp = _dev(loss, "loss") if loss is not None else None
        return B, lw, lp

    def train_step(self, x: torch.Tensor, t: torch.Tensor, loss_weights, lr: float,
                   loss: Optional[torch.Tensor] = None, stream=None):
        B, lw, lp = self._train_args(x, t, loss_weights, loss)
        _check(load().sgrid_mlp_train_step(self.handle, _dev(x, "x"), _dev(t, "t"), B, lw.ctypes.data_as(_P),
                                           float(lr), lp, _stream(stream)))

    def apply_gradient(self, grad: torch.Tensor, lr: float, stream=None):
        """One Adam step from a caller's gradient [44804] (FP32, device)."""
        _f32(grad, "grad", MLP_N_PARAMS)
        _check(load().sgrid_mlp_apply_gradient(self.handle, _dev(grad, "grad"), float(lr), _stream(stream)))


def gather_windows(grid: Grid, phi: torch.Tensor, x: Optional[torch.Tensor] = None,
                   unsat: Optional[torch.Tensor] = None, stream=None):
    """Windows of phi/h [n_core*64, 216] and unsaturated flags [n_core*64] of the core points."""
    n = grid.n_core * 64
    _f32(phi, "phi", grid.n_total * 64)
    if x is not None and (x.shape != (n, 216) or x.dtype != torch.float32):
        raise ValueError("x must be [n_core*64, 216] float32")
    if unsat is not None and (unsat.numel() != n or unsat.dtype != torch.uint8):
        raise ValueError("unsat must be [n_core*64] uint8")
    _check(load().sgrid_gather_windows(grid.handle, _dev(phi, "phi"), _dev(x, "x") if x is not None else None,
                                       _dev(unsat, "unsat") if unsat is not None else None, _stream(stream)))


class Batch:
    """Many grids swept together; fields are the grids' fields concatenated."""

    def __init__(self, grids, stream=None):
        import numpy as np
        self.grids = list(grids)
        arr = (_P * len(self.grids))(*[g.handle for g in self.grids])
        out = ctypes.c_void_p()
        _check(load().sgrid_batch_create(arr, len(self.grids), _stream(stream), ctypes.byref(out)))
        self._h = out
        nt, nw = ctypes.c_int64(), ctypes.c_int64()
        bases = np.zeros(len(self.grids), dtype=np.int64)
        _check(load().sgrid_batch_info(self._h, ctypes.byref(nt), ctypes.byref(nw), bases.ctypes.data_as(_P)))
        self.n_total, self.n_work, self.bases = int(nt.value), int(nw.value), bases

    @property
    def handle(self):
        if self._h is None:
            raise SgridError(5, "batch already destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _check(load().sgrid_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_config(self, variant: int, blocks_per_cu: int):
        _check(load().sgrid_batch_set_config(self.handle, int(variant), int(blocks_per_cu)))

    def autotune(self, phi: torch.Tensor, scratch: torch.Tensor, reps: int = 10, stream=None):
        """Returns (variant, blocks_per_cu, table[2][6] of us per sweep for
        blocks_per_cu in (1, 2, 4, 8, 16, 0))."""
        import numpy as np
        _f32(phi, "phi", self.n_total * 64)
        _f32(scratch, "scratch", self.n_total * 64)
        v, b = ctypes.c_int32(), ctypes.c_int32()
        table = np.zeros(12, dtype=np.float32)
        _check(load().sgrid_batch_autotune(self.handle, _dev(phi, "phi"), _dev(scratch, "scratch"), int(reps),
                                           _stream(stream), ctypes.byref(v), ctypes.byref(b),
                                           table.ctypes.data_as(_P)))
        return int(v.value), int(b.value), table.reshape(2, 6)

    def reinitialize(self, phi: torch.Tensor, scratch: torch.Tensor, n_iter: int, use_graph: bool = True,
                     stream=None):
        _f32(phi, "phi", self.n_total * 64)
        _f32(scratch, "scratch", self.n_total * 64)
        _check(load().sgrid_batch_reinitialize(self.handle, _dev(phi, "phi"), _dev(scratch, "scratch"),
                                               int(n_iter), int(bool(use_graph)), _stream(stream)))


SWEEP_TUNE_CANDIDATES = ((0, 1), (0, 2), (2, 4), (3, 1), (3, 2), (5, 1), (7, 1))


def autotune_sweep(grid: "Grid", phi: torch.Tensor, scratch: torch.Tensor, reps: int = 10, stream=None):
    """Times the sweep candidates on this grid (phi is read, scratch written),
    makes the fastest the configuration and returns (variant, groups, us per
    sweep for each of SWEEP_TUNE_CANDIDATES)."""
    import numpy as np
    if scratch.dtype != phi.dtype or scratch.numel() != phi.numel() or phi.numel() != grid.n_total * 64:
        raise ValueError("phi and scratch must both be [P+2, 64] of one dtype")
    v, g = ctypes.c_int32(), ctypes.c_int32()
    table = np.zeros(len(SWEEP_TUNE_CANDIDATES), dtype=np.float32)
    _check(load().sgrid_autotune_sweep(grid.handle, _dtype_code(phi), _dev(phi, "phi"), _dev(scratch, "scratch"),
                                       int(reps), _stream(stream), ctypes.byref(v), ctypes.byref(g),
                                       table.ctypes.data_as(_P)))
    return int(v.value), int(g.value), table


def set_sweep_config(variant: int, groups: int):
    """Select the sweep kernel variant (0 = DPP exchange, 1 = LDS tile) and the
    number of four-package sets each wavefront processes."""
    _check(load().sgrid_set_sweep_config(int(variant), int(groups)))
