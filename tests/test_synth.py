"""Pins of the synthetic input generators (analytic signed distances, noise,
particles) against hand-derived values."""
import math

import numpy as np

import synth


def test_splitmix64_published_vectors():
    # Sequence of SplitMix64 from state 0 (the generator adds the golden gamma
    # before mixing): the first outputs as published with the algorithm.
    out = synth.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_noise_range_and_determinism():
    lin = np.arange(100000)
    u = synth.unit_noise(3, lin)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01
    assert np.array_equal(u[500:600], synth.unit_noise(3, lin[500:600]))
    assert not np.array_equal(u, synth.unit_noise(4, lin))


def test_sphere_and_box():
    s = synth.sphere()
    assert synth.sdf(s, [[0.5, 0.5, 0.5]])[0] == -0.3
    assert abs(synth.sdf(s, [[0.8, 0.5, 0.5]])[0]) < 1e-15
    b = synth.box((0.5, 0.5, 0.5), (0.2, 0.1, 0.3))
    assert abs(synth.sdf(b, [[0.5, 0.5, 0.5]])[0] + 0.1) < 1e-15
    assert abs(synth.sdf(b, [[0.8, 0.5, 0.5]])[0] - 0.1) < 1e-15               # face
    assert abs(synth.sdf(b, [[0.8, 0.7, 0.5]])[0] - math.hypot(0.1, 0.1)) < 1e-15  # edge
    assert abs(synth.sdf(b, [[0.8, 0.7, 0.9]])[0] - math.sqrt(0.03)) < 1e-15     # corner


def test_prism():
    p = synth.prism()
    # centroid at (0.5, 0.5): inradius of an equilateral triangle of side a is a / (2 sqrt 3)
    inr = 0.6 / (2 * math.sqrt(3))
    assert abs(synth.sdf(p, [[0.5, 0.5, 0.5]])[0] + inr) < 1e-15
    # below the bottom edge (horizontal, at y = 0.5 - inr)
    assert abs(synth.sdf(p, [[0.5, 0.5 - inr - 0.05, 0.5]])[0] - 0.05) < 1e-14
    # above the top vertex (0.5, 0.5 + 2 inr)
    assert abs(synth.sdf(p, [[0.5, 0.5 + 2 * inr + 0.07, 0.5]])[0] - 0.07) < 1e-14
    # beyond the end caps (z = 0.1 and 0.9)
    assert abs(synth.sdf(p, [[0.5, 0.5, 0.95]])[0] - 0.05) < 1e-14
    # near a cap, inside: the cap is closer than the sides
    assert abs(synth.sdf(p, [[0.5, 0.5, 0.88]])[0] + 0.02) < 1e-14
    # outside both a side and a cap: Euclidean combination
    assert abs(synth.sdf(p, [[0.5, 0.5 - inr - 0.03, 0.94]])[0] - 0.05) < 1e-14


def test_torus_and_displacement():
    t = synth.torus()
    for th in np.linspace(0, 2 * math.pi, 7):
        x = [0.5 + 0.35 * math.cos(th), 0.5 + 0.35 * math.sin(th), 0.5]
        assert abs(synth.sdf(t, [x])[0] + 0.1) < 1e-15
    d = synth.displaced_torus(7)
    assert abs(sum(abs(a) for a in d["a"]) - 1.0) < 1e-12
    pts = synth.surface_particles(d, 2000, 1, 0.0).astype(np.float64)
    # sampled points lie on the displaced surface up to the first-order normal offset
    assert np.abs(synth.sdf(d, pts)).max() < 5e-3


def test_particles():
    s = synth.sphere()
    p = synth.shell_particles(20000, 1, s["center"], 0.28, 0.32)
    r = np.linalg.norm(p.astype(np.float64) - 0.5, axis=1)
    assert p.dtype == np.float32 and r.min() >= 0.28 - 1e-6 and r.max() <= 0.32 + 1e-6
    q = synth.surface_particles(synth.prism(), 20000, 2, 0.0).astype(np.float64)
    assert np.abs(synth.sdf(synth.prism(), q)).max() < 1e-6
