"""Seeded synthetic inputs for the narrow-band sparse-grid workloads.

This module is shared by the GPU path's tests and benchmark *and* by the CPU
oracle, so it deliberately holds no step of the sparse-grid method itself (no
activation, numbering, neighbour lookup, reinitialisation, differencing,
interpolation or integral).  It only produces inputs:

* analytic signed-distance functions (sphere, box, triangular prism, torus,
  displaced torus, unions) evaluated in float64;
* a counter-based per-data-point noise value, so that any subset of the fine
  grid (a package, an oracle crop) can be regenerated independently;
* particle positions (uniform in a shell, or area-uniform on a surface plus
  Gaussian jitter), rounded to float32 once so that both sides consume the
  same values.

Coordinates: the domain is the unit cube with origin 0.  A fine grid of N
points per axis has spacing h = 1/N and its data point (i, j, k) sits at the
fine-cell centre ((i, j, k) + 1/2) * h.  Coarse (background) cells have size
4h; coarse cell (a, b, c) has centre ((a, b, c) + 1/2) * 4h.  Linear indices
run x fastest.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Sequence

import numpy as np


__all__ = [
    "splitmix64", "unit_noise", "sdf", "coarse_sdf", "fine_points",
    "phi0_at", "sphere", "box", "prism", "torus", "displaced_torus", "union",
    "random_union", "batch_shapes", "shell_particles", "surface_particles",
    "config_c1", "config_c2", "config_c3", "config_c5", "config_shell", "shell",
]

def _threads() -> int:
    """Worker threads for chunked evaluation (numpy releases the GIL in its
    array kernels, so chunks run in parallel)."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n or (os.cpu_count() or 1)))


def _chunked(n: int, chunk: int, fn):
    """Calls fn(start, stop) over [0, n) in chunks on a thread pool."""
    starts = list(range(0, n, chunk))
    if len(starts) <= 1:
        for a in starts:
            fn(a, min(a + chunk, n))
        return
    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        list(ex.map(lambda a: fn(a, min(a + chunk, n)), starts))


# ---------------------------------------------------------------------------
# Counter-based noise: SplitMix64 (Steele, Lea & Flood, "Fast splittable
# pseudorandom number generators", OOPSLA 2014), used as a hash of a 64-bit key.
# ---------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(key: np.ndarray) -> np.ndarray:
    """SplitMix64 output for each 64-bit key (the generator's state after one
    increment by the golden gamma, then the published finaliser)."""
    z = np.asarray(key, dtype=np.uint64) + _GOLDEN
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def unit_noise(seed: int, lin: np.ndarray) -> np.ndarray:
    """u in [-1, 1) for fine linear index `lin` under `seed`.

    key = seed * 2^40 + lin (lin < 2^40 covers grids up to 8192^3); the top 53
    bits of SplitMix64(key) give v in [0, 1) exactly; u = 2v - 1."""
    key = (np.uint64(seed) << np.uint64(40)) + np.asarray(lin, dtype=np.uint64)
    top = splitmix64(key) >> np.uint64(11)
    return top.astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


# ---------------------------------------------------------------------------
# Analytic signed distances (negative inside).  Shapes are plain dicts so that
# they serialise into benchmark records.
# ---------------------------------------------------------------------------

def sphere(center=(0.5, 0.5, 0.5), radius=0.3) -> Dict:
    return {"kind": "sphere", "center": list(map(float, center)), "radius": float(radius)}


def shell(center=(0.5, 0.5, 0.5), r_in=0.3, r_out=0.31) -> Dict:
    """Spherical shell r_in <= |x - center| <= r_out (negative inside the shell)."""
    return {"kind": "shell", "center": list(map(float, center)), "r_in": float(r_in), "r_out": float(r_out)}


def box(center=(0.5, 0.5, 0.5), half=(0.2, 0.2, 0.2)) -> Dict:
    return {"kind": "box", "center": list(map(float, center)), "half": list(map(float, half))}


def prism(edge=0.6, length=0.8, center=(0.5, 0.5, 0.5)) -> Dict:
    """Equilateral triangle of side `edge` in the xy-plane, centroid at
    (center.x, center.y), one vertex towards +y, extruded over `length`
    along z about center.z."""
    return {"kind": "prism", "edge": float(edge), "length": float(length),
            "center": list(map(float, center))}


def torus(center=(0.5, 0.5, 0.5), R=0.35, r=0.1) -> Dict:
    """Torus with axis z through `center`, tube centre-line radius R, tube radius r."""
    return {"kind": "torus", "center": list(map(float, center)), "R": float(R), "r": float(r)}


def displaced_torus(seed: int, center=(0.5, 0.5, 0.5), R=0.35, r=0.1,
                    amplitude=0.02, n_modes=8) -> Dict:
    """Torus whose surface is displaced by amplitude * sum_k a_k sin(m_k theta
    + n_k varphi + psi_k) with integer m_k in [1, 8], n_k in [1, 4], psi_k
    uniform in [0, 2 pi) and sum |a_k| = 1 (so |displacement| <= amplitude)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 9, size=n_modes)
    n = rng.integers(1, 5, size=n_modes)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    a = rng.uniform(-1.0, 1.0, size=n_modes)
    a = a / np.abs(a).sum()
    return {"kind": "displaced_torus", "center": list(map(float, center)), "R": float(R),
            "r": float(r), "amplitude": float(amplitude), "m": m.tolist(), "n": n.tolist(),
            "psi": psi.tolist(), "a": a.tolist()}


def union(parts: Sequence[Dict]) -> Dict:
    return {"kind": "union", "parts": list(parts)}


def _tri_vertices(s: Dict) -> np.ndarray:
    cx, cy, _ = s["center"]
    rc = s["edge"] / math.sqrt(3.0)  # circumradius
    ang = np.array([90.0, 210.0, 330.0]) * math.pi / 180.0
    return np.stack([cx + rc * np.cos(ang), cy + rc * np.sin(ang)], axis=1)


def _triangle_sdf2(px: np.ndarray, py: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Exact 2D signed distance to a counter-clockwise triangle."""
    d2 = np.full(px.shape, np.inf)
    inside = np.ones(px.shape, dtype=bool)
    for e in range(3):
        ax, ay = v[e]
        bx, by = v[(e + 1) % 3]
        ex, ey = bx - ax, by - ay
        wx, wy = px - ax, py - ay
        t = np.clip((wx * ex + wy * ey) / (ex * ex + ey * ey), 0.0, 1.0)
        dx, dy = wx - t * ex, wy - t * ey
        d2 = np.minimum(d2, dx * dx + dy * dy)
        inside &= (ex * wy - ey * wx) > 0.0  # left of every CCW edge
    d = np.sqrt(d2)
    return np.where(inside, -d, d)


def _torus_angles(s: Dict, x: np.ndarray):
    c = np.asarray(s["center"])
    dx, dy, dz = x[:, 0] - c[0], x[:, 1] - c[1], x[:, 2] - c[2]
    rho = np.hypot(dx, dy)
    theta = np.arctan2(dy, dx)
    varphi = np.arctan2(dz, rho - s["R"])
    return rho, dz, theta, varphi


def _displacement(s: Dict, theta: np.ndarray, varphi: np.ndarray) -> np.ndarray:
    out = np.zeros_like(theta)
    for a, m, n, psi in zip(s["a"], s["m"], s["n"], s["psi"]):
        out += a * np.sin(m * theta + n * varphi + psi)
    return s["amplitude"] * out


def sdf(s: Dict, x: np.ndarray) -> np.ndarray:
    """Signed distance of shape `s` at points x[n, 3] (float64)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    k = s["kind"]
    if k == "sphere":
        return np.linalg.norm(x - np.asarray(s["center"]), axis=1) - s["radius"]
    if k == "shell":
        r = np.linalg.norm(x - np.asarray(s["center"]), axis=1)
        return np.maximum(r - s["r_out"], s["r_in"] - r)
    if k == "box":
        q = np.abs(x - np.asarray(s["center"])) - np.asarray(s["half"])
        outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
        return outside + np.minimum(q.max(axis=1), 0.0)
    if k == "prism":
        d2 = _triangle_sdf2(x[:, 0], x[:, 1], _tri_vertices(s))
        dz = np.abs(x[:, 2] - s["center"][2]) - 0.5 * s["length"]
        w0, w1 = d2, dz
        return np.minimum(np.maximum(w0, w1), 0.0) + np.hypot(np.maximum(w0, 0.0), np.maximum(w1, 0.0))
    if k == "torus":
        rho, dz, _, _ = _torus_angles(s, x)
        return np.hypot(rho - s["R"], dz) - s["r"]
    if k == "displaced_torus":
        rho, dz, theta, varphi = _torus_angles(s, x)
        return np.hypot(rho - s["R"], dz) - s["r"] - _displacement(s, theta, varphi)
    if k == "union":
        out = sdf(s["parts"][0], x)
        for p in s["parts"][1:]:
            out = np.minimum(out, sdf(p, x))
        return out
    raise ValueError(f"unknown shape kind {k!r}")


# ---------------------------------------------------------------------------
# Grid sampling
# ---------------------------------------------------------------------------

def coarse_sdf(s: Dict, n_coarse: int, chunk: int = 1 << 20, origin=(0, 0, 0),
               extent: int | None = None) -> np.ndarray:
    """float32 signed distance at coarse-cell centres, x fastest, evaluated in
    float64 and rounded once to float32.

    With the defaults it covers the whole M^3 background grid (shape (M^3,)).
    `origin` and `extent` select the sub-box of extent^3 coarse cells starting
    at coarse cell `origin` (cell size still 1/M), for crops of large grids."""
    M = int(n_coarse)
    E = M if extent is None else int(extent)
    o = np.asarray(origin, dtype=np.int64)
    lc = 1.0 / M
    out = np.empty(E ** 3, dtype=np.float32)

    def work(a, b):
        lin = np.arange(a, b, dtype=np.int64)
        i, j, k = lin % E + o[0], (lin // E) % E + o[1], lin // (E * E) + o[2]
        x = (np.stack([i, j, k], axis=1).astype(np.float64) + 0.5) * lc
        out[a:b] = sdf(s, x).astype(np.float32)

    _chunked(E ** 3, chunk, work)
    return out


def child_sdf(s: Dict, parents: np.ndarray, M: int, chunk: int = 1 << 18) -> np.ndarray:
    """float32 signed distance at the centres of the eight children of each
    coarse cell in `parents` (linear indices on the M^3 grid) on the grid of
    doubled resolution (2M)^3; shape (n, 8), child b = bx + 2 by + 4 bz,
    evaluated in float64 and rounded once (the values the dense (2M)^3
    sampling gives at those cells)."""
    parents = np.asarray(parents, dtype=np.int64)
    n = parents.shape[0]
    out = np.empty((n, 8), dtype=np.float32)
    b = np.arange(8)
    off = np.stack([b & 1, (b >> 1) & 1, (b >> 2) & 1], axis=1)

    def work(a, e):
        c = parents[a:e]
        ijk = np.stack([c % M, (c // M) % M, c // (M * M)], axis=1)
        f = 2 * ijk[:, None, :] + off[None, :, :]
        x = (f.reshape(-1, 3).astype(np.float64) + 0.5) / (2 * M)
        out[a:e] = sdf(s, x).astype(np.float32).reshape(-1, 8)

    _chunked(n, chunk, work)
    return out


def fine_points(lin: np.ndarray, N: int) -> np.ndarray:
    """Positions ((i, j, k) + 1/2) h of fine linear indices `lin` on an N^3 grid."""
    lin = np.asarray(lin, dtype=np.int64)
    i, j, k = lin % N, (lin // N) % N, lin // (N * N)
    return (np.stack([i, j, k], axis=1).astype(np.float64) + 0.5) / N


def phi0_at(s: Dict, N: int, lin: np.ndarray, noise_amp: float, noise_seed: int,
            chunk: int = 1 << 20) -> np.ndarray:
    """Initial level-set values (float64) at fine linear indices `lin`:
    sdf(x) * (1 + noise_amp * u(seed, lin)).  The multiplicative form keeps the
    sign and the zero set of the signed distance."""
    lin = np.asarray(lin, dtype=np.int64).ravel()
    out = np.empty(lin.shape[0], dtype=np.float64)

    def work(a, b):
        l = lin[a:b]
        v = sdf(s, fine_points(l, N))
        if noise_amp != 0.0:
            v = v * (1.0 + noise_amp * unit_noise(noise_seed, l))
        out[a:b] = v

    _chunked(lin.shape[0], chunk, work)
    return out


# ---------------------------------------------------------------------------
# Batches of random unions (many shapes, uneven sizes)
# ---------------------------------------------------------------------------

def random_union(rng: np.random.Generator) -> Dict:
    """Union of 1-4 primitives with centres U[0.3, 0.7]^3: spheres r~U[0.05, 0.25],
    boxes half-extents ~U[0.05, 0.2]^3, tori R~U[0.1, 0.2], r~U[0.03, 0.08]."""
    parts = []
    for _ in range(int(rng.integers(1, 5))):
        kind = int(rng.integers(0, 3))
        c = rng.uniform(0.3, 0.7, size=3)
        if kind == 0:
            parts.append(sphere(c, rng.uniform(0.05, 0.25)))
        elif kind == 1:
            parts.append(box(c, rng.uniform(0.05, 0.2, size=3)))
        else:
            parts.append(torus(c, rng.uniform(0.1, 0.2), rng.uniform(0.03, 0.08)))
    return union(parts)


def batch_shapes(n_shapes: int, seed: int, resolutions=(64, 128, 256, 512)) -> List[Dict]:
    """`n_shapes` seeded random unions, each with a fine resolution drawn
    uniformly from `resolutions`; returned as dicts with keys shape, N, noise_seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_shapes):
        shp = random_union(rng)
        N = int(rng.choice(np.asarray(resolutions)))
        out.append({"shape": shp, "N": N, "noise_seed": int(seed * 1000 + i + 1)})
    return out


# ---------------------------------------------------------------------------
# Particles
# ---------------------------------------------------------------------------

def shell_particles(n: int, seed: int, center, r_in: float, r_out: float) -> np.ndarray:
    """n points uniform in the spherical shell r_in <= |x - center| <= r_out, float32."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = np.cbrt(r_in ** 3 + rng.uniform(0.0, 1.0, n) * (r_out ** 3 - r_in ** 3))
    return (np.asarray(center) + d * rad[:, None]).astype(np.float32)


def _prism_surface(s: Dict, n: int, rng) -> np.ndarray:
    v = _tri_vertices(s)
    e, L = s["edge"], s["length"]
    zc = s["center"][2]
    a_cap = math.sqrt(3.0) / 4.0 * e * e
    areas = np.array([a_cap, a_cap, e * L, e * L, e * L])
    face = rng.choice(5, size=n, p=areas / areas.sum())
    out = np.empty((n, 3))
    # caps: uniform in the triangle via folded barycentrics
    u1, u2 = rng.uniform(size=n), rng.uniform(size=n)
    fold = u1 + u2 > 1.0
    u1, u2 = np.where(fold, 1.0 - u1, u1), np.where(fold, 1.0 - u2, u2)
    capx = v[0, 0] + u1 * (v[1, 0] - v[0, 0]) + u2 * (v[2, 0] - v[0, 0])
    capy = v[0, 1] + u1 * (v[1, 1] - v[0, 1]) + u2 * (v[2, 1] - v[0, 1])
    t, w = rng.uniform(size=n), rng.uniform(-0.5, 0.5, size=n)
    for f in range(5):
        m = face == f
        if f < 2:
            out[m, 0], out[m, 1] = capx[m], capy[m]
            out[m, 2] = zc + (0.5 * L if f == 0 else -0.5 * L)
        else:
            a, b = v[f - 2], v[(f - 1) % 3]
            out[m, 0] = a[0] + t[m] * (b[0] - a[0])
            out[m, 1] = a[1] + t[m] * (b[1] - a[1])
            out[m, 2] = zc + w[m] * L
    return out


def _torus_surface(s: Dict, n: int, rng) -> np.ndarray:
    """Area-uniform points on a torus (rejection on the tube angle)."""
    R, r = s["R"], s["r"]
    c = np.asarray(s["center"])
    pts = []
    need = n
    while need > 0:
        m = int(need * (R + r) / R) + 16
        th = rng.uniform(0.0, 2 * math.pi, m)
        ph = rng.uniform(0.0, 2 * math.pi, m)
        keep = rng.uniform(0.0, R + r, m) < R + r * np.cos(ph)
        th, ph = th[keep][:need], ph[keep][:need]
        rho = R + r * np.cos(ph)
        p = np.stack([rho * np.cos(th), rho * np.sin(th), r * np.sin(ph)], axis=1) + c
        if s["kind"] == "displaced_torus":
            delta = _displacement(s, th, ph)
            nrm = np.stack([np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph)], axis=1)
            p = p + delta[:, None] * nrm
        pts.append(p)
        need -= len(th)
    return np.concatenate(pts)[:n]


def surface_particles(s: Dict, n: int, seed: int, sigma: float, chunk: int = 1 << 20) -> np.ndarray:
    """n points area-uniform on the surface of `s` plus isotropic N(0, sigma^2 I)
    jitter, float32.  Supports prisms, spheres and (displaced) tori.  Chunk c
    of `chunk` points draws from the generator seeded with (seed, c), so the
    set does not depend on how many threads produce it."""
    out = np.empty((n, 3), dtype=np.float32)

    def work(a, b):
        rng = np.random.default_rng([seed, a // chunk])
        m = b - a
        if s["kind"] == "prism":
            p = _prism_surface(s, m, rng)
        elif s["kind"] in ("torus", "displaced_torus"):
            p = _torus_surface(s, m, rng)
        elif s["kind"] == "sphere":
            d = rng.standard_normal((m, 3))
            p = np.asarray(s["center"]) + s["radius"] * d / np.linalg.norm(d, axis=1, keepdims=True)
        else:
            raise ValueError(f"surface sampling not provided for {s['kind']!r}")
        out[a:b] = (p + sigma * rng.standard_normal((m, 3))).astype(np.float32)

    _chunked(n, chunk, work)
    return out


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def config_c1() -> Dict:
    """Sphere r=0.3 centred in the unit cube, 64^3 data points, noise 10%,
    20 reinitialisation iterations, 1e5 particles uniform in the band."""
    return {"name": "sphere64", "shape": sphere(), "N": 64, "noise_amp": 0.1, "noise_seed": 1,
            "n_iter": 20, "n_particles": 100_000, "particle_seed": 2, "particles": "shell"}


def config_c2() -> Dict:
    """Extruded triangular prism (edge 0.6, extrusion 0.8), 512^3 data points,
    noise 5%, 100 iterations, 1e7 particles jittered N(0, 0.5h) about the surface."""
    return {"name": "prism512", "shape": prism(), "N": 512, "noise_amp": 0.05, "noise_seed": 3,
            "n_iter": 100, "n_particles": 10_000_000, "particle_seed": 4, "particles": "surface"}


def config_c3(n_shapes=64, seed=5) -> Dict:
    """64 seeded random unions at resolutions from {64, 128, 256, 512}^3,
    noise 10%, 50 iterations."""
    return {"name": "batch64", "shapes": batch_shapes(n_shapes, seed), "noise_amp": 0.1, "n_iter": 50}


def config_c5() -> Dict:
    """Displaced torus R=0.35, r=0.1 at 2048^3, 100 iterations, 5e7 particles."""
    return {"name": "torus2048", "shape": displaced_torus(7), "N": 2048, "noise_amp": 0.0,
            "noise_seed": 0, "n_iter": 100, "n_particles": 50_000_000, "particle_seed": 8,
            "particles": "surface"}


def config_shell() -> Dict:
    """The paper's timing geometry (Sec. 9, Tab. 1): shell of radii 0.3 and 0.31
    about (0.5, 0.5, 0.5) at resolution 1/1024; phi0 is its signed distance."""
    return {"name": "shell1024", "shape": shell(), "N": 1024, "noise_amp": 0.0, "noise_seed": 0,
            "delta": 1.0e-6}


def particles_for(cfg: Dict, n: int | None = None) -> np.ndarray:
    """Particle positions of a named workload (float32, shape (n, 3))."""
    n = cfg["n_particles"] if n is None else int(n)
    h = 1.0 / cfg["N"]
    s = cfg["shape"]
    if cfg["particles"] == "shell":
        w = 2 * 4 * h
        return shell_particles(n, cfg["particle_seed"], s["center"], s["radius"] - w, s["radius"] + w)
    return surface_particles(s, n, cfg["particle_seed"], 0.5 * h)
