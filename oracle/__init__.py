"""Plain FP64 CPU oracle for the narrow-band sparse-grid hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library; the arithmetic lives in `oracle.c` (plain loops on a
dense N^3 grid, double precision) and this module only marshals numpy arrays.

Dense conventions: N = 4M data points per axis, data point (i, j, k) at
((i, j, k) + 1/2) h, linear index i + N j + N^2 k.  Points of cells that are
not activated hold the far-field constant of their cell, -B inside and +B
outside, with B = 16 h; reads outside the domain return +B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

N_PARAM = 44804


def build() -> str:
    """Compile oracle.c with gcc (OpenMP, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_DEFAULT_SOURCE",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "orc_classify": (None, [i32, f64, P, P]),
            "orc_correct_signs": (i32, [i32, f64, P, P]),
            "orc_correct_point_signs": (i32, [i32, P, i64, P, P]),
            "orc_number": (i64, [i32, P, P, P, P, P]),
            "orc_neighbours": (None, [i32, P, P, i64, P]),
            "orc_index_shift": (None, [i32, P, P]),
            "orc_reinit": (None, [i32, f64, f64, P, i64, P, P, i32]),
            "orc_gradient": (None, [i32, f64, f64, P, i64, P, P, P, P]),
            "orc_laplacian": (None, [i32, f64, f64, P, i64, P, P]),
            "orc_probe": (None, [i32, f64, f64, P, P, P, P, P, P, i64, P, P, P]),
            "orc_probe_field": (None, [i32, f64, P, P, P, P, i64, P]),
            "orc_plane_cube_fraction": (f64, [f64, f64, f64, f64]),
            "orc_wendland": (f64, [f64]),
            "orc_wendland_dr": (f64, [f64]),
            "orc_support_offsets": (i32, [P]),
            "orc_integrals": (None, [i32, f64, f64, P, P, i64, P]),
            "orc_windows": (None, [i32, f64, f64, P, P, i64, P]),
            "orc_mlp_n_params": (i32, []),
            "orc_gelu": (f64, [f64]),
            "orc_gelu_grad": (f64, [f64]),
            "orc_mlp_forward": (None, [P, P, i64, P]),
            "orc_mlp_backward": (None, [P, P, P, i64, P]),
            "orc_adam": (None, [i64, P, P, P, P, i64, f64, f64, f64, f64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Tables
# --------------------------------------------------------------------------

def classify(M: int, lc: float, d: np.ndarray) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float32)
    t = np.zeros(M ** 3, dtype=np.uint8)
    lib().orc_classify(M, lc, _p(d), _p(t))
    return t


def correct_signs(M: int, d: np.ndarray, lc: Optional[float] = None):
    """Sign correction of coarse distances d[M^3] by diffusion from the core
    cells (Sec. 7.2, coarse step); returns (corrected d, rounds)."""
    d = np.ascontiguousarray(d, dtype=np.float32)
    lc = 1.0 / M if lc is None else float(lc)
    out = np.empty_like(d)
    rounds = int(lib().orc_correct_signs(M, lc, _p(d), _p(out)))
    return out, rounds


def correct_point_signs(N: int, tab: "Tables", phi: np.ndarray):
    """Sign correction of the inner packages' data points by diffusion from the
    core packages and the far field (Sec. 7.2, refined step); phi is the dense
    state (far-field constants outside the band).  Returns (corrected dense
    phi, rounds)."""
    inner = active_points(tab, pkg_types=(2,))
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    if phi.shape != (N ** 3,):
        raise ValueError(f"phi must be the dense field of N^3 = {N ** 3} values")
    out = np.empty_like(phi)
    rounds = int(lib().orc_correct_point_signs(N, _p(inner), inner.shape[0], _p(phi), _p(out)))
    return out, rounds


@dataclass
class Tables:
    M: int
    cell_type: np.ndarray   # u8[M^3]
    cell_pkg: np.ndarray    # u32[M^3]
    pkg_cell: np.ndarray    # u32[P+2]
    pkg_type: np.ndarray    # u8[P+2]
    nbr: np.ndarray         # u32[P+2, 27]

    @property
    def n_packages(self) -> int:
        return int(self.pkg_cell.shape[0]) - 2


def build_tables(M: int, d: np.ndarray, lc: Optional[float] = None) -> Tables:
    """Activation, numbering and neighbour table for coarse distances d[M^3]
    with coarse cell size `lc` (default 1/M, the unit cube; a crop of a larger
    grid passes that grid's cell size)."""
    d = np.ascontiguousarray(d, dtype=np.float32)
    lc = 1.0 / M if lc is None else float(lc)
    t = classify(M, lc, d)
    n = M ** 3
    cell_pkg = np.zeros(n, dtype=np.uint32)
    pkg_cell = np.zeros(n + 2, dtype=np.uint32)
    pkg_type = np.zeros(n + 2, dtype=np.uint8)
    P = int(lib().orc_number(M, _p(d), _p(t), _p(cell_pkg), _p(pkg_cell), _p(pkg_type)))
    pkg_cell = pkg_cell[:P + 2].copy()
    pkg_type = pkg_type[:P + 2].copy()
    nbr = np.zeros((P + 2, 27), dtype=np.uint32)
    lib().orc_neighbours(M, _p(cell_pkg), _p(pkg_cell), P + 2, _p(nbr))
    return Tables(M, t, cell_pkg, pkg_cell, pkg_type, nbr)


def refine_tables(M: int, d: np.ndarray, child_d: np.ndarray):
    """The next layer of the multi-resolution construction (Sec. 7, Sec. 7.1
    step 1): the layer of doubled resolution (2M)^3 whose distances are
    evaluated only in the cells covered by core cells of the layer with
    distances d[M^3].
    child_d[i, b] is the distance at child b = bx + 2 by + 4 bz of the i-th
    core cell in ascending cell order.  Every other fine cell carries its
    parent's distance, which is at least the parent's cell size in magnitude
    (the parent is not core) and so never tags it core, and gives it the
    parent's sign.  Then tagging, numbering and neighbours as for any layer.
    Returns the tables and the distances the layer holds per cell (the input
    of the next refinement)."""
    d = np.ascontiguousarray(d, dtype=np.float32)
    child_d = np.ascontiguousarray(child_d, dtype=np.float32).reshape(-1, 8)
    Mf = 2 * M
    t = classify(M, 1.0 / M, d)
    core = np.nonzero(t == 1)[0]
    if core.shape[0] != child_d.shape[0]:
        raise ValueError(f"{core.shape[0]} core cells but {child_d.shape[0]} rows of child distances")
    slot = np.full(M ** 3, -1, dtype=np.int64)
    slot[core] = np.arange(core.shape[0])
    f = np.arange(Mf ** 3, dtype=np.int64)
    fi, fj, fk = f % Mf, (f // Mf) % Mf, f // (Mf * Mf)
    parent = (fi // 2) + M * ((fj // 2) + M * (fk // 2))
    child = (fi & 1) + 2 * (fj & 1) + 4 * (fk & 1)
    sp = slot[parent]
    del fi, fj, fk
    under = sp >= 0
    d_f = d[parent]
    d_f[under] = child_d[sp[under], child[under]]
    return build_tables(Mf, d_f), d_f


def index_shift(s: int):
    slot, data = ctypes.c_int32(), ctypes.c_int32()
    lib().orc_index_shift(int(s), ctypes.byref(slot), ctypes.byref(data))
    return slot.value, data.value


# --------------------------------------------------------------------------
# Dense state
# --------------------------------------------------------------------------

def active_points(tab: Tables, pkg_types=(1, 2)) -> np.ndarray:
    """Fine linear indices of every data point of activated cells of the given
    types, ascending."""
    M = tab.M
    N = 4 * M
    cells = np.nonzero(np.isin(tab.cell_type, np.asarray(pkg_types, dtype=np.uint8)))[0].astype(np.int64)
    cx, cy, cz = cells % M, (cells // M) % M, cells // (M * M)
    loc = np.arange(64, dtype=np.int64)
    lx, ly, lz = loc % 4, (loc // 4) % 4, loc // 16
    i = (4 * cx)[:, None] + lx[None, :]
    j = (4 * cy)[:, None] + ly[None, :]
    k = (4 * cz)[:, None] + lz[None, :]
    return np.sort((i + N * (j + N * k)).ravel())


def dense_state(tab: Tables, active: np.ndarray, phi0_active: np.ndarray, B: float) -> np.ndarray:
    """Dense N^3 float64 field: phi0 at the active points, the far-field
    constant of their cell elsewhere (-B for package 0, +B for package 1)."""
    M = tab.M
    N = 4 * M
    far = np.where(tab.cell_pkg == 0, -B, B).astype(np.float64).reshape(M, M, M)
    phi = np.repeat(np.repeat(np.repeat(far, 4, axis=0), 4, axis=1), 4, axis=2).reshape(-1)
    phi[active] = phi0_active
    assert phi.shape[0] == N ** 3
    return phi


def reinit(N: int, h: float, B: float, active: np.ndarray, phi: np.ndarray, n_iter: int) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64).copy()
    work = np.empty_like(phi)
    act = np.ascontiguousarray(active, dtype=np.int64)
    lib().orc_reinit(N, h, B, _p(act), act.shape[0], _p(phi), _p(work), n_iter)
    return phi


def gradient(N: int, h: float, B: float, active: np.ndarray, phi: np.ndarray):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    g = np.zeros((3, N ** 3), dtype=np.float64)
    act = np.ascontiguousarray(active, dtype=np.int64)
    lib().orc_gradient(N, h, B, _p(act), act.shape[0], _p(phi), _p(g[0]), _p(g[1]), _p(g[2]))
    return g


def laplacian(N: int, h: float, B: float, active: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Seven-point Laplacian at the active points of a dense field (0 elsewhere):
    the stencil operation of the paper's timing test (Sec. 9, Tab. 1)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(N ** 3, dtype=np.float64)
    act = np.ascontiguousarray(active, dtype=np.int64)
    lib().orc_laplacian(N, h, B, _p(act), act.shape[0], _p(phi), _p(out))
    return out


def sequential_update(phi: np.ndarray, active: np.ndarray, delta: float) -> np.ndarray:
    """The sequential operation of the paper's timing test (Sec. 9, Tab. 1): a
    small change to every active value, here phi + delta."""
    out = np.array(phi, dtype=np.float64, copy=True)
    out[active] += delta
    return out


def probe(N: int, h: float, B: float, cell_pkg: np.ndarray, phi: np.ndarray, g: np.ndarray,
          pos: np.ndarray, with_gradient: bool = False):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    out = np.empty(n, dtype=np.float64)
    nrm = np.empty((n, 3), dtype=np.float64)
    gout = np.empty((n, 3), dtype=np.float64) if with_gradient else None
    cp = np.ascontiguousarray(cell_pkg, dtype=np.uint32)
    lib().orc_probe(N, h, B, _p(cp), _p(np.ascontiguousarray(phi)), _p(np.ascontiguousarray(g[0])),
                    _p(np.ascontiguousarray(g[1])), _p(np.ascontiguousarray(g[2])),
                    _p(pos), n, _p(out), _p(nrm), _p(gout) if with_gradient else None)
    return (out, nrm, gout) if with_gradient else (out, nrm)


def c_full() -> float:
    """K_W of a support wholly on the phi > 0 side: the sum of the 32 kernel
    weights of the dual-cell query (8 taps at sqrt(3)/2 h, 24 at sqrt(11)/2 h)."""
    return 8.0 * wendland(0.5 * np.sqrt(3.0)) + 24.0 * wendland(0.5 * np.sqrt(11.0))


def integral_field(N: int, h: float, B: float, tab: Tables, active: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Dense [4][N^3] integral field (Sec. 8): the integrals at every
    activated point; every other point holds the constants of its cell's
    far-field package, (0, 0, 0, 0) inside and (c_full, 0, 0, 0) outside."""
    f = np.zeros((4, N ** 3), dtype=np.float64)
    M = N // 4
    cp = np.asarray(tab.cell_pkg)
    i = np.arange(N, dtype=np.int64)
    jj, ii = np.meshgrid(i, i, indexing="ij")                    # one z-layer, x fastest
    layer = (ii // 4) + M * (jj // 4)
    c = c_full()
    for k in range(N):                                            # layer by layer: no N^3 index arrays
        f[0, k * N * N:(k + 1) * N * N] = np.where(cp[layer.ravel() + M * M * (k // 4)] == 1, c, 0.0)
    act = np.asarray(active, dtype=np.int64)
    f[:, act] = integrals(N, h, B, phi, act).T
    return f


def probe_field(N: int, h: float, cell_pkg: np.ndarray, f: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of the dense [4][N^3] integral field at the
    particles ([n][4]), with the probe's corner rules; a particle whose home
    cell is far field takes that package's constants."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    far = np.array([[0.0, 0.0, 0.0, 0.0], [c_full(), 0.0, 0.0, 0.0]])
    out = np.empty((pos.shape[0], 4), dtype=np.float64)
    lib().orc_probe_field(N, h, _p(np.ascontiguousarray(cell_pkg, dtype=np.uint32)),
                          _p(np.ascontiguousarray(f, dtype=np.float64)), _p(far), _p(pos), pos.shape[0], _p(out))
    return out


def plane_cube_fraction(a: float, g) -> float:
    return lib().orc_plane_cube_fraction(float(a), float(g[0]), float(g[1]), float(g[2]))


def wendland(r: float) -> float:
    return lib().orc_wendland(float(r))


def wendland_dr(r: float) -> float:
    return lib().orc_wendland_dr(float(r))


def support_offsets() -> np.ndarray:
    off = np.zeros((64, 3), dtype=np.int32)
    n = lib().orc_support_offsets(_p(off))
    return off[:n].copy()


def integrals(N: int, h: float, B: float, phi: np.ndarray, pts: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    if phi.shape != (N ** 3,):
        raise ValueError(f"phi must be the dense field of N^3 = {N ** 3} values")
    out = np.empty((pts.shape[0], 4), dtype=np.float64)
    lib().orc_integrals(N, h, B, _p(phi), _p(pts),
                        pts.shape[0], _p(out))
    return out


def windows(N: int, h: float, B: float, phi: np.ndarray, pts: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty((pts.shape[0], 216), dtype=np.float64)
    lib().orc_windows(N, h, B, _p(np.ascontiguousarray(phi, dtype=np.float64)), _p(pts),
                      pts.shape[0], _p(out))
    return out


# --------------------------------------------------------------------------
# MLP
# --------------------------------------------------------------------------

def gelu(z: float) -> float:
    return lib().orc_gelu(float(z))


def gelu_grad(z: float) -> float:
    return lib().orc_gelu_grad(float(z))


def mlp_forward(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 216)
    y = np.empty((x.shape[0], 4), dtype=np.float64)
    lib().orc_mlp_forward(_p(w), _p(x), x.shape[0], _p(y))
    return y


def mlp_backward(w: np.ndarray, x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 216)
    dy = np.ascontiguousarray(dy, dtype=np.float64).reshape(-1, 4)
    dw = np.empty(N_PARAM, dtype=np.float64)
    lib().orc_mlp_backward(_p(w), _p(x), _p(dy), x.shape[0], _p(dw))
    return dw


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays w, m, v."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_adam(w.shape[0], _p(w), _p(g), _p(m), _p(v), int(t), lr, beta1, beta2, eps)


# --------------------------------------------------------------------------
# One whole plain pass of a workload on the dense grid
# --------------------------------------------------------------------------

@dataclass
class DenseRun:
    N: int
    h: float
    B: float
    tab: Tables
    active: np.ndarray
    phi0: np.ndarray        # phi0 at `active` (float64 values as consumed)
    phi: Optional[np.ndarray] = None      # dense after reinitialisation
    grad: Optional[np.ndarray] = None     # dense [3, N^3]


def setup(shape, N: int, noise_amp: float, noise_seed: int, phi0_dtype=np.float32) -> DenseRun:
    """Coarse distances, tables and phi0 for a shape; phi0 is rounded to
    `phi0_dtype` (the precision the GPU path consumes) and upcast exactly."""
    import synth
    M = N // 4
    h = 1.0 / N
    d = synth.coarse_sdf(shape, M)
    tab = build_tables(M, d)
    act = active_points(tab)
    phi0 = synth.phi0_at(shape, N, act, noise_amp, noise_seed).astype(phi0_dtype).astype(np.float64)
    return DenseRun(N, h, 16.0 * h, tab, act, phi0)


@dataclass
class CropRun(DenseRun):
    origin: tuple = (0, 0, 0)     # first coarse cell of the crop in the full grid
    n_full: int = 0               # data points per axis of the full grid


def setup_crop(shape, N: int, origin, extent: int, noise_amp: float, noise_seed: int,
               phi0_dtype=np.float32) -> CropRun:
    """The dense oracle state of a sub-box of a grid too large to hold whole:
    extent^3 coarse cells starting at coarse cell `origin` of the N^3 grid, with
    the full grid's spacing, far-field constant and initial values.  Inside the
    crop everything is local: N of the returned run is 4 extent.

    Every update reads face neighbours only, so after n iterations (and one
    gradient) a crop point whose distance to every crop face exceeds n plus the
    reach of activation (one coarse cell) holds exactly the value the full grid
    computes there; points nearer the faces see the crop's edge as far field."""
    import synth
    M = N // 4
    o = tuple(int(v) for v in origin)
    assert all(0 <= v and v + extent <= M for v in o)
    h = 1.0 / N
    d = synth.coarse_sdf(shape, M, origin=o, extent=extent)
    tab = build_tables(extent, d, lc=1.0 / M)
    act = active_points(tab)
    n = 4 * extent
    i, j, k = act % n + 4 * o[0], (act // n) % n + 4 * o[1], act // (n * n) + 4 * o[2]
    glob = i + N * (j + N * k)
    phi0 = synth.phi0_at(shape, N, glob, noise_amp, noise_seed).astype(phi0_dtype).astype(np.float64)
    return CropRun(n, h, 16.0 * h, tab, act, phi0, origin=o, n_full=N)


def run_plain(run: DenseRun, n_iter: int) -> DenseRun:
    phi = dense_state(run.tab, run.active, run.phi0, run.B)
    run.phi = reinit(run.N, run.h, run.B, run.active, phi, n_iter)
    run.grad = gradient(run.N, run.h, run.B, run.active, run.phi)
    return run
