"""Pins of the oracle's near-surface kernel integrals (Sec. 8 names the
integral with an SPH smoothing kernel; the definition follows the reading
the design document states: dual-cell query point, Wendland C2 kernel with
smoothing length h and support 2h, exact plane-cube cut fractions).

Independent anchors: quadrature of the kernel (normalisation), finite
differences (kernel derivative), Monte Carlo / midpoint sampling and
elementary closed forms (plane-cube fraction), brute-force enumeration
(support set), and symmetries (complement, reflection, permutation).
"""
import itertools

import numpy as np
import pytest
from scipy import integrate

import oracle

# --- kernel ---------------------------------------------------------------

def test_wendland_normalised_and_compact():
    val, _ = integrate.quad(lambda r: 4 * np.pi * r * r * oracle.wendland(r), 0, 2, epsabs=1e-14)
    assert abs(val - 1.0) < 1e-12
    assert oracle.wendland(2.0) == 0.0 and oracle.wendland(2.5) == 0.0
    assert oracle.wendland(0.0) == pytest.approx(21 / (16 * np.pi))


def test_wendland_derivative_matches_finite_difference():
    for r in np.linspace(0.05, 1.95, 39):
        e = 1e-6
        fd = (oracle.wendland(r + e) - oracle.wendland(r - e)) / (2 * e)
        assert abs(fd - oracle.wendland_dr(r)) < 1e-8


def test_support_offsets_brute_force():
    off = oracle.support_offsets()
    expect = []
    for oz, oy, ox in itertools.product(range(-3, 5), repeat=3):
        r2 = (ox - 0.5) ** 2 + (oy - 0.5) ** 2 + (oz - 0.5) ** 2
        if r2 < 4.0:
            expect.append((ox, oy, oz))
    assert sorted(map(tuple, off.tolist())) == sorted(expect)
    r2 = ((off - 0.5) ** 2).sum(axis=1)
    assert len(off) == 32 and (r2 == 0.75).sum() == 8 and (r2 == 2.75).sum() == 24
    # offsets stay within {-1..2}, so central differences need the 6^3 window {-2..3}
    assert off.min() == -1 and off.max() == 2


# --- plane-cube fraction ---------------------------------------------------

def test_plane_cube_fraction_monte_carlo():
    rng = np.random.default_rng(1)
    u = rng.uniform(-0.5, 0.5, (400_000, 3))
    for _ in range(40):
        g = rng.standard_normal(3) * rng.choice([0.1, 1.0, 5.0])
        a = rng.uniform(-1.0, 1.0) * (np.abs(g).sum() / 2 + 0.1)
        mc = np.mean(a + u @ g > 0)
        assert abs(oracle.plane_cube_fraction(a, g) - mc) < 4e-3


def test_plane_cube_fraction_midpoint_grid_nearly_aligned():
    # Nearly axis-aligned normals (two tiny components) are where closed forms
    # cancel badly; compare with a fine midpoint rule.
    n = 200
    c = (np.arange(n) + 0.5) / n - 0.5
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    for g, a in [((1.0, 1e-9, 2e-9), 0.1), ((1e-7, 1.0, 1e-7), -0.3), ((3e-8, 2e-8, 2.0), 0.05),
                 ((0.7, 0.3, 1e-10), 0.2)]:
        mid = np.mean(a + g[0] * X + g[1] * Y + g[2] * Z > 0)
        assert abs(oracle.plane_cube_fraction(a, g) - mid) < 1e-4
    # a diagonal edge with a vanishing third component: the excluded region
    # u1 + u2 <= -a/0.7 is a right triangle at the corner with legs 1 - a/0.7
    L = 1.0 - 0.2 / 0.7
    assert oracle.plane_cube_fraction(0.2, (0.7, 0.7, 1e-10)) == pytest.approx(1 - L * L / 2, abs=1e-9)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_cube_fraction_axis_aligned_is_ramp(axis):
    for a in np.linspace(-0.8, 0.8, 33):
        for s in (0.5, 1.0, 2.0, -1.0):
            g = [0.0, 0.0, 0.0]
            g[axis] = s
            expect = min(max(0.5 + a / abs(s), 0.0), 1.0)
            assert oracle.plane_cube_fraction(a, g) == pytest.approx(expect, abs=1e-14)


def test_plane_cube_fraction_corner_tetrahedron_and_symmetries():
    rng = np.random.default_rng(2)
    for _ in range(50):
        m = rng.uniform(0.2, 2.0, 3)
        alpha = rng.uniform(0, 0.9) * m.min()
        # region g.u > c near the corner u = (1/2,1/2,1/2): volume alpha^3 / (6 m1 m2 m3)
        a = alpha - m.sum() / 2
        assert oracle.plane_cube_fraction(a, m) == pytest.approx(alpha ** 3 / (6 * m.prod()), rel=1e-12)
        g = rng.standard_normal(3)
        aa = rng.uniform(-1, 1)
        v = oracle.plane_cube_fraction(aa, g)
        assert oracle.plane_cube_fraction(-aa, -g) == pytest.approx(1 - v, abs=1e-14)
        for perm in itertools.permutations(range(3)):
            assert oracle.plane_cube_fraction(aa, g[list(perm)]) == pytest.approx(v, abs=1e-14)
        assert oracle.plane_cube_fraction(aa, g * [-1, 1, 1]) == pytest.approx(v, abs=1e-14)
    assert oracle.plane_cube_fraction(0.0, [0, 0, 0]) == 0.5
    assert oracle.plane_cube_fraction(1e-3, [0, 0, 0]) == 1.0
    assert oracle.plane_cube_fraction(-1e-3, [0, 0, 0]) == 0.0


# --- integrals on small dense grids -----------------------------------------

N = 16
H = 1.0 / N
B = 16 * H


def _coords():
    i = np.arange(N ** 3)
    return (np.stack([i % N, (i // N) % N, i // (N * N)], axis=1) + 0.5) * H


def _pts(margin=4):
    x = _coords()
    idx = np.nonzero(np.all((x > margin * H) & (x < 1 - margin * H), axis=1))[0]
    return idx.astype(np.int64)


def _C():
    off = oracle.support_offsets()
    r = np.sqrt(((off - 0.5) ** 2).sum(axis=1))
    return sum(oracle.wendland(v) for v in r)


def test_integrals_full_and_empty():
    pts = _pts()
    full = oracle.integrals(N, H, B, np.full(N ** 3, 5 * H), pts)
    assert np.allclose(full[:, 0], _C(), atol=1e-14)
    assert np.allclose(full[:, 1:], 0.0, atol=1e-14)
    empty = oracle.integrals(N, H, B, np.full(N ** 3, -5 * H), pts)
    assert np.all(empty == 0.0)


def test_integrals_plane_through_query_is_half():
    # phi = x - q_x for every query: V_j pairs up as (V, 1 - V) symmetrically.
    x = _coords()
    pts = _pts()[:50]
    for p in pts:
        q = x[p] + 0.5 * H
        phi = x[:, 0] - q[0]
        out = oracle.integrals(N, H, B, phi, np.array([p]))
        assert out[0, 0] == pytest.approx(_C() / 2, abs=1e-14)
        assert out[0, 1] > 0.5                 # kernel gradient points to the phi > 0 side
        assert abs(out[0, 2]) < 1e-14 and abs(out[0, 3]) < 1e-14


def test_integrals_antisymmetry_reflection_permutation():
    rng = np.random.default_rng(4)
    x = _coords()
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    phi = (x - 0.5) @ n + 0.3 * np.sin(7 * x[:, 0]) * H + rng.uniform(-0.3, 0.3, N ** 3) * H
    pts = _pts()
    base = oracle.integrals(N, H, B, phi, pts)
    assert np.abs(base[:, 0]).max() > 0.05
    neg = oracle.integrals(N, H, B, -phi, pts)
    assert np.allclose(neg[:, 0], _C() - base[:, 0], atol=1e-13)
    assert np.allclose(neg[:, 1:], -base[:, 1:], atol=1e-13)
    # reflect x: the query point of p maps to the query point of the mirrored
    # data point p' = N-2-i (the dual cell between i and i+1 maps to the one
    # between N-2-i and N-1-i), so compare through that map.
    f = phi.reshape(N, N, N)
    fr = np.ascontiguousarray(f[:, :, ::-1]).ravel()
    i, j, k = pts % N, (pts // N) % N, pts // (N * N)
    mp = (N - 2 - i) + N * (j + N * k)
    refl = oracle.integrals(N, H, B, fr, mp)
    assert np.allclose(refl[:, 0], base[:, 0], atol=1e-13)
    assert np.allclose(refl[:, 1], -base[:, 1], atol=1e-13)
    assert np.allclose(refl[:, 2:], base[:, 2:], atol=1e-13)
    # swap x and y: outputs 1 and 2 swap
    fs = np.ascontiguousarray(f.transpose(0, 2, 1)).ravel()
    sp = j + N * (i + N * k)
    sw = oracle.integrals(N, H, B, fs, sp)
    assert np.allclose(sw[:, 0], base[:, 0], atol=1e-13)
    assert np.allclose(sw[:, 1], base[:, 2], atol=1e-13)
    assert np.allclose(sw[:, 2], base[:, 1], atol=1e-13)
    assert np.allclose(sw[:, 3], base[:, 3], atol=1e-13)


def test_integrals_axis_plane_uses_ramp_fractions():
    # phi = x - d: central differences give g = (1,0,0) exactly, so every V_j is
    # the ramp clamp(1/2 + phi_j/h); the sum is then an explicit finite sum.
    x = _coords()
    p = _pts()[100]
    q = x[p] + 0.5 * H
    off = oracle.support_offsets()
    for d_over_h in (0.0, 0.25, 0.5, -0.25, 0.9):
        phi = x[:, 0] - (q[0] + d_over_h * H)
        out = oracle.integrals(N, H, B, phi, np.array([p]))[0]
        kw, kg = 0.0, np.zeros(3)
        for o in off:
            xj = x[p] + o * H
            V = min(max(0.5 + (xj[0] - q[0]) / H - d_over_h, 0.0), 1.0)
            dv = (q - xj) / H
            r = np.linalg.norm(dv)
            kw += oracle.wendland(r) * V
            kg += oracle.wendland_dr(r) * dv / r * V
        assert out[0] == pytest.approx(kw, abs=1e-14)
        assert np.allclose(out[1:], kg, atol=1e-14)


def test_windows_layout():
    x = _coords()
    rng = np.random.default_rng(9)
    phi = rng.standard_normal(N ** 3)
    pts = _pts()[:20]
    w = oracle.windows(N, H, B, phi, pts)
    for q, p in enumerate(pts):
        i, j, k = p % N, (p // N) % N, p // (N * N)
        cube = phi.reshape(N, N, N)[k - 2:k + 4, j - 2:j + 4, i - 2:i + 4]
        assert np.array_equal(w[q], cube.ravel() / H)
