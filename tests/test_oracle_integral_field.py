"""Pins of the oracle's integral field and its particle probe (Sec. 8):
one-sided supports, exact recovery at data points, exact reproduction of
linear fields by the trilinear blend, the far-field home rule, and agreement
with the phi/gradient probe, which blends the same corners by its own code."""
import numpy as np
import pytest

import oracle



def _all_active_cell_pkg(M):
    return (2 + np.arange(M ** 3)).astype(np.uint32)


def test_c_full_is_the_one_sided_integral():
    # a field positive everywhere: every cut fraction is 1, so K_W is the sum
    # of the kernel weights and K_grad vanishes by symmetry
    N, h, B = 16, 1.0 / 16, 1.0
    phi = np.full(N ** 3, 0.5)
    pts = np.array([5 + N * (6 + N * 7)], dtype=np.int64)
    k = oracle.integrals(N, h, B, phi, pts)[0]
    assert abs(k[0] - oracle.c_full()) <= 1e-14
    assert np.all(np.abs(k[1:]) <= 1e-14)
    # and negative everywhere: nothing on the phi > 0 side
    k = oracle.integrals(N, h, B, -phi, pts)[0]
    assert np.all(np.abs(k) <= 1e-15)
    # a discrete sum of a unit-integral kernel over 32 of the 64 nearest points
    assert 0.95 < oracle.c_full() < 1.0


def test_probe_field_recovers_data_points():
    N, h = 16, 1.0 / 16
    rng = np.random.default_rng(3)
    f = rng.standard_normal((4, N ** 3))
    ijk = rng.integers(0, N, (300, 3))
    pos = (ijk + 0.5) * h
    out = oracle.probe_field(N, h, _all_active_cell_pkg(N // 4), f, pos)
    lin = ijk[:, 0] + N * (ijk[:, 1] + N * ijk[:, 2])
    assert np.allclose(out, f[:, lin].T, rtol=0, atol=1e-14)


def test_probe_field_reproduces_linear_fields():
    N, h = 16, 1.0 / 16
    p = np.arange(N ** 3)
    x = np.stack([(p % N + 0.5) * h, ((p // N) % N + 0.5) * h, (p // (N * N) + 0.5) * h])
    a = np.array([[0.3, 1.0, -2.0, 0.5], [-1.0, 0.0, 0.7, 2.0], [0.1, -0.4, 0.0, 1.5], [2.0, 0.2, 0.3, -0.6]])
    f = a[:, :1] + a[:, 1:] @ x
    rng = np.random.default_rng(4)
    pos = rng.uniform(0.5 * h, 1 - 0.5 * h, (500, 3))       # inside the hull of the data points
    out = oracle.probe_field(N, h, _all_active_cell_pkg(N // 4), f, pos)
    want = (a[:, :1] + a[:, 1:] @ pos.T).T
    assert np.allclose(out, want, rtol=0, atol=1e-13)


def test_probe_field_far_field_home():
    N, h = 16, 1.0 / 16
    M = N // 4
    cp = _all_active_cell_pkg(M)
    cp[0] = 0                   # cell (0, 0, 0): negative far field
    cp[M ** 3 - 1] = 1          # cell (M-1, M-1, M-1): positive far field
    f = np.random.default_rng(5).standard_normal((4, N ** 3))
    pos = np.array([[0.01, 0.02, 0.2 * h], [1 - 0.01, 1 - 0.3 * h, 0.99], [1.5, 1.2, 2.0], [-1.0, -0.5, -0.1]])
    out = oracle.probe_field(N, h, cp, f, pos)
    c = oracle.c_full()
    assert np.all(out[0] == 0.0) and np.all(out[3] == 0.0)      # clamped into cell (0, 0, 0)
    assert out[1, 0] == c and np.all(out[1, 1:] == 0.0)
    assert out[2, 0] == c and np.all(out[2, 1:] == 0.0)


def test_probe_field_matches_the_phi_probe_blend():
    N, h, B = 16, 1.0 / 16, 1.0
    rng = np.random.default_rng(6)
    f = rng.standard_normal((4, N ** 3))
    pos = rng.uniform(-0.05, 1.05, (400, 3))
    cp = _all_active_cell_pkg(N // 4)
    out = oracle.probe_field(N, h, cp, f, pos)
    v, _, g = oracle.probe(N, h, B, cp, f[0], f[1:], pos, with_gradient=True)
    assert np.allclose(out[:, 0], v, rtol=0, atol=1e-14)
    assert np.allclose(out[:, 1:], g, rtol=0, atol=1e-14)


def test_integral_field_dense_layout():
    # a small band: activated points carry the integrals, every other point
    # the constants of its cell's far-field package
    import synth
    N = 32
    M, h = N // 4, 1.0 / N
    run = oracle.setup(synth.sphere((0.5, 0.5, 0.5), 0.3), N, 0.1, 2)
    oracle.run_plain(run, 3)
    f = oracle.integral_field(run.N, run.h, run.B, run.tab, run.active, run.phi)
    act = np.zeros(N ** 3, dtype=bool)
    act[run.active] = True
    p = np.arange(N ** 3)
    cell = (p % N) // 4 + M * (((p // N) % N) // 4 + M * ((p // (N * N)) // 4))
    side = np.asarray(run.tab.cell_pkg)[cell]
    c = oracle.c_full()
    assert np.all(f[0, ~act & (side == 0)] == 0.0) and np.all(f[0, ~act & (side == 1)] == c)
    assert np.all(f[1:, ~act] == 0.0)
    k = oracle.integrals(run.N, h, run.B, run.phi, run.active[:50])
    assert np.array_equal(f[:, run.active[:50]].T, k)
