"""Pins of the oracle's field operations: upwind reinitialisation, central
difference (Sec. 7.3, Listing 5) and trilinear probing (Sec. 8).

Expected values are closed forms (fixed points, one-step constant-field
update, exactness on polynomial fields) or symmetries that a wrong sign,
swapped branch, wrong axis or wrong index would break.
"""
import numpy as np
import pytest

import oracle
import synth

N = 16
H = 1.0 / N
B = 16 * H


def _grid():
    i = np.arange(N ** 3)
    x = (np.stack([i % N, (i // N) % N, i // (N * N)], axis=1) + 0.5) * H
    return i.astype(np.int64), x


def _interior(x, margin):
    lo, hi = margin * H, 1.0 - margin * H
    return np.all((x > lo) & (x < hi), axis=1)


@pytest.mark.parametrize("seed", range(4))
def test_reinit_linear_field_is_fixed_point(seed):
    # Any linear field with unit gradient satisfies |grad phi| = 1 exactly under
    # one-sided differences, so the upwind update leaves it unchanged.
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    act, x = _grid()
    phi = x @ n - 0.5 * n.sum() + rng.uniform(-0.1, 0.1)
    out = oracle.reinit(N, H, B, act, phi, 3)
    inner = _interior(x, 4)
    assert np.max(np.abs(out[inner] - phi[inner])) < 1e-14


@pytest.mark.parametrize("c", [0.3 * H, -0.7 * H, 2.5 * H, -4.0 * H])
def test_reinit_constant_field_one_step(c):
    # Zero gradient: phi' = c - (h/2) S (0 - 1) = c + (h/2) c / sqrt(c^2 + h^2).
    act, x = _grid()
    phi = np.full(N ** 3, c)
    out = oracle.reinit(N, H, B, act, phi, 1)
    inner = _interior(x, 1)
    expect = c + 0.5 * H * c / np.sqrt(c * c + H * H)
    assert np.allclose(out[inner], expect, rtol=0, atol=1e-15)


def _kink(axis, c, sign, offset):
    """phi = sign * (|x_axis - x_c| + offset) on the all-active grid: a field
    of unit slope on both sides of the data-point plane x_axis = x_c, which
    is a ridge (sign < 0 after the shift) or a valley (sign > 0)."""
    act, x = _grid()
    xc = (c + 0.5) * H
    return act, x, sign * (np.abs(x[:, axis] - xc) + offset), np.isclose(x[:, axis], xc)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_reinit_kink_one_step_closed_form(axis, sign):
    # Valley phi = |x - c| + h/2 (and its negative).  Away from the kink plane
    # the field is linear with unit slope, so every branch gives G = 1 and the
    # point is fixed.  On the plane D- = -1 and D+ = +1 (times the sign): the
    # upwind branch of the sign of phi takes neither difference (both point
    # away from the upwind side), G = 0, and the point moves by dt |S| in the
    # direction of its sign, with S = (h/2) / sqrt(h^2/4 + h^2) = 1/sqrt(5).
    # The downwind choice would take both, G = 1, and leave the point fixed.
    act, x, phi, on = _kink(axis, 7, sign, 0.5 * H)
    out = oracle.reinit(N, H, B, act, phi, 1)
    inner = _interior(x, 1)
    expect = phi.copy()
    expect[on] = sign * (0.5 * H + 0.5 * H / np.sqrt(5.0))
    assert on[inner].sum() == (N - 2) ** 2
    assert np.max(np.abs(out[inner] - expect[inner])) < 1e-15


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_reinit_ridge_is_stationary(axis, sign):
    # Ridge phi = -|x - c| + 2.5h (and its negative): on the ridge plane the
    # upwind branch takes both one-sided differences (each points towards the
    # surface), G = 1, and the point is fixed; every other point lies on a
    # unit-slope linear piece (no data point sits on phi = 0, which is 2.5h
    # from the plane).  The downwind choice would give G = 0 and move the
    # ridge by dt S.
    act, x, phi, on = _kink(axis, 8, -sign, -2.5 * H)
    out = oracle.reinit(N, H, B, act, phi, 1)
    inner = _interior(x, 1)
    assert not np.any(phi == 0.0)
    assert np.max(np.abs(out[inner] - phi[inner])) < 1e-15


def test_reinit_zero_is_stationary():
    act, x = _grid()
    out = oracle.reinit(N, H, B, act, np.zeros(N ** 3), 2)
    assert np.all(out[_interior(x, 2)] == 0.0)


def test_reinit_antisymmetry_and_axis_equivariance():
    rng = np.random.default_rng(7)
    act, x = _grid()
    phi = rng.uniform(-3 * H, 3 * H, N ** 3)
    n_it = 2
    out = oracle.reinit(N, H, B, act, phi, n_it)
    inner = _interior(x, n_it + 1)
    # phi -> -phi gives -result away from the (positive) out-of-domain padding
    neg = oracle.reinit(N, H, B, act, -phi, n_it)
    assert np.allclose(neg[inner], -out[inner], atol=1e-15)
    # permuting axes permutes the result; reflecting an axis reflects it
    f = phi.reshape(N, N, N)
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0)]:
        g = np.ascontiguousarray(f.transpose(perm)).ravel()
        og = oracle.reinit(N, H, B, act, g, n_it).reshape(N, N, N)
        back = np.ascontiguousarray(og.transpose(np.argsort(perm))).ravel()
        assert np.allclose(back[inner], out[inner], atol=1e-15)
    for ax in range(3):
        g = np.ascontiguousarray(np.flip(f, axis=ax)).ravel()
        og = np.flip(oracle.reinit(N, H, B, act, g, n_it).reshape(N, N, N), axis=ax).ravel()
        assert np.allclose(og[inner], out[inner], atol=1e-15)


def test_reinit_far_field_points_untouched():
    rng = np.random.default_rng(3)
    act, x = _grid()
    phi = rng.uniform(-2 * H, 2 * H, N ** 3)
    sub = act[::3]
    out = oracle.reinit(N, H, B, sub, phi, 4)
    mask = np.ones(N ** 3, dtype=bool)
    mask[sub] = False
    assert np.array_equal(out[mask], phi[mask])


def test_reinit_noisy_sphere_converges_to_distance():
    # Sanity (not an exact pin): 64^3 sphere with 10% multiplicative noise;
    # after 20 iterations the band near the surface is close to the distance
    # and |grad phi| is close to 1.
    cfg = synth.config_c1()
    run = oracle.setup(cfg["shape"], 64, 0.1, 1, phi0_dtype=np.float64)
    before = np.abs(run.phi0 - synth.sdf(cfg["shape"], synth.fine_points(run.active, 64)))
    oracle.run_plain(run, 20)
    sd = synth.sdf(cfg["shape"], synth.fine_points(run.active, 64))
    near = np.abs(sd) < 2 * run.h
    err = np.abs(run.phi[run.active] - sd)
    assert err[near].max() < 0.2 * run.h
    # the multiplicative noise grows with distance; the iteration removes most of it
    band = (np.abs(sd) >= 2 * run.h) & (np.abs(sd) < 8 * run.h)
    assert err[band].mean() < 0.6 * before[band].mean()
    g = run.grad[:, run.active]
    gn = np.linalg.norm(g, axis=0)
    mid = np.abs(sd) < 4 * run.h
    assert np.median(np.abs(gn[mid] - 1)) < 0.02


def test_gradient_exact_on_quadratics():
    rng = np.random.default_rng(11)
    act, x = _grid()
    A = rng.standard_normal((3, 3))
    A = A + A.T
    b = rng.standard_normal(3)
    phi = 0.5 * np.einsum("ni,ij,nj->n", x, A, x) + x @ b
    g = oracle.gradient(N, H, B, act, phi)
    inner = _interior(x, 1)
    exact = x @ A + b  # A symmetric
    assert np.max(np.abs(g[:, inner].T - exact[inner])) < 1e-12
    # points not listed as active keep a zero gradient
    g2 = oracle.gradient(N, H, B, act[:10], phi)
    assert np.all(g2[:, 10:] == 0)


def _probe_setup(M=4):
    """An all-active coarse grid (every distance 0)."""
    d = np.zeros(M ** 3, dtype=np.float32)
    tab = oracle.build_tables(M, d)
    Nn = 4 * M
    i = np.arange(Nn ** 3)
    x = (np.stack([i % Nn, (i // Nn) % Nn, i // (Nn * Nn)], axis=1) + 0.5) / Nn
    return tab, Nn, x


def test_probe_exact_on_trilinear_fields():
    tab, Nn, x = _probe_setup()
    h = 1.0 / Nn
    rng = np.random.default_rng(5)
    c = rng.standard_normal(8)

    def f(p):
        X, Y, Z = p[:, 0], p[:, 1], p[:, 2]
        return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * Y + c[5] * Y * Z
                + c[6] * X * Z + c[7] * X * Y * Z)

    phi = f(x)
    g = np.stack([f(x) * 0 + c[1] + c[4] * x[:, 1] + c[6] * x[:, 2] + c[7] * x[:, 1] * x[:, 2],
                  c[2] + c[4] * x[:, 0] + c[5] * x[:, 2] + c[7] * x[:, 0] * x[:, 2],
                  c[3] + c[5] * x[:, 1] + c[6] * x[:, 0] + c[7] * x[:, 0] * x[:, 1]])
    pos = rng.uniform(0.5 * h, 1 - 0.5 * h, (2000, 3))
    val, nrm = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, phi, g, pos)
    assert np.max(np.abs(val - f(pos))) < 1e-12
    # the gradient fields are trilinear too, so the interpolated g is exact
    gx = c[1] + c[4] * pos[:, 1] + c[6] * pos[:, 2] + c[7] * pos[:, 1] * pos[:, 2]
    gy = c[2] + c[4] * pos[:, 0] + c[5] * pos[:, 2] + c[7] * pos[:, 0] * pos[:, 2]
    gz = c[3] + c[5] * pos[:, 1] + c[6] * pos[:, 0] + c[7] * pos[:, 0] * pos[:, 1]
    ge = np.stack([gx, gy, gz], axis=1)
    assert np.allclose(nrm, ge / np.linalg.norm(ge, axis=1, keepdims=True), atol=1e-12)


def test_probe_returns_data_values_and_constants():
    tab, Nn, x = _probe_setup()
    h = 1.0 / Nn
    rng = np.random.default_rng(6)
    phi = rng.standard_normal(Nn ** 3)
    g = rng.standard_normal((3, Nn ** 3))
    pick = rng.choice(Nn ** 3, 500)
    val, nrm = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, phi, g, x[pick])
    assert np.array_equal(val, phi[pick])
    gp = g[:, pick].T
    assert np.allclose(nrm, gp / np.linalg.norm(gp, axis=1, keepdims=True), atol=1e-14)
    # constant field: weights sum to one, zero gradient gives a zero normal
    val, nrm = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, np.full(Nn ** 3, 0.25), np.zeros((3, Nn ** 3)),
                            rng.uniform(-0.1, 1.1, (500, 3)))
    assert np.allclose(val, 0.25, atol=1e-15, rtol=0) and np.all(nrm == 0)


def test_probe_continuous_across_cell_faces():
    tab, Nn, x = _probe_setup()
    h = 1.0 / Nn
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(Nn ** 3)
    g = rng.standard_normal((3, Nn ** 3))
    face = (rng.integers(1, Nn - 1, (300, 3)) + 0.5) * h  # data-point planes
    face[:, 1:] += rng.uniform(-0.4, 0.4, (300, 2)) * h
    eps = 1e-9
    a, _ = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, phi, g, face - [eps, 0, 0])
    b, _ = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, phi, g, face + [eps, 0, 0])
    assert np.max(np.abs(a - b)) < 1e-6


def test_probe_far_field_home_cell():
    # Only the centre cell of a 5^3 coarse grid is core (its 26 neighbours are
    # inner); particles in corner cells see the far-field constant of their own
    # cell and a zero normal.
    M = 5
    d = np.full(M ** 3, 5.0, dtype=np.float32)
    d[62] = 0.0
    d[0] = -5.0
    tab = oracle.build_tables(M, d)
    assert tab.n_packages == 27 and tab.cell_type[62] == 1
    Nn = 20
    h = 1.0 / Nn
    phi = np.full(Nn ** 3, 99.0)
    g = np.ones((3, Nn ** 3))
    pos = np.array([[0.1, 0.1, 0.1], [0.9, 0.9, 0.9], [0.5, 0.5, 0.5]])
    val, nrm = oracle.probe(Nn, h, 16 * h, tab.cell_pkg, phi, g, pos)
    assert val[0] == -16 * h and val[1] == 16 * h and abs(val[2] - 99.0) < 1e-12
    assert np.all(nrm[:2] == 0)


# --------------------------------------------------------------------------
# The operations of the paper's timing test (Sec. 9, Tab. 1)
# --------------------------------------------------------------------------

def test_laplacian_exact_on_quadratics():
    # The seven-point stencil is exact for quadratics: sum of 2 a_ii for any
    # mixed and linear terms, here with dyadic coefficients so FP64 is exact.
    act, x = _grid()
    c = x - 0.5
    phi = 0.75 * c[:, 0] ** 2 - 1.25 * c[:, 1] ** 2 + 2.5 * c[:, 2] ** 2 + 0.5 * c[:, 0] * c[:, 1] - c[:, 2] + 0.125
    lap = oracle.laplacian(N, H, B, act, phi)
    inner = _interior(x, 1)
    assert np.max(np.abs(lap[inner] - 2 * (0.75 - 1.25 + 2.5))) < 1e-9
    assert np.max(np.abs(oracle.laplacian(N, H, B, act, x @ np.array([0.3, -0.2, 0.7]))[inner])) < 1e-9


def test_laplacian_brute_force_with_far_field():
    # Against a padded numpy evaluation on a band that leaves far-field cells:
    # the active list from the tables, every other point holding +-B.
    s = synth.sphere((0.5, 0.5, 0.5), 0.3)
    run = oracle.setup(s, N, 0.1, 3, phi0_dtype=np.float64)
    phi = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    lap = oracle.laplacian(N, H, B, run.active, phi)
    P = np.pad(phi.reshape(N, N, N), 1, constant_values=B)
    c = P[1:-1, 1:-1, 1:-1]
    ref = (P[1:-1, 1:-1, :-2] + P[1:-1, 1:-1, 2:] + P[1:-1, :-2, 1:-1] + P[1:-1, 2:, 1:-1]
           + P[:-2, 1:-1, 1:-1] + P[2:, 1:-1, 1:-1] - 6 * c) / H ** 2
    mask = np.zeros(N ** 3, dtype=bool)
    mask[run.active] = True
    assert np.allclose(lap[mask], ref.ravel()[mask], rtol=1e-13, atol=1e-9)
    assert np.all(lap[~mask] == 0.0)
    # some active points see the far field across a face
    assert (np.abs(ref.ravel()[mask]) > 100).any()


def test_sequential_update():
    act, x = _grid()
    phi = np.sin(x[:, 0] * 7)
    sel = act[::3]
    out = oracle.sequential_update(phi, sel, 1e-3)
    assert np.array_equal(out[sel], phi[sel] + 1e-3)
    rest = np.setdiff1d(act, sel)
    assert np.array_equal(out[rest], phi[rest])
