"""Pins of the oracle's surrogate network (216 -> 128 -> 128 -> 4, tanh GELU)
and its Adam update: finite differences, the closed-form first Adam step, and
the known gap between the tanh and erf forms of GELU."""
import math

import numpy as np
import pytest

import oracle


def _params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(oracle.N_PARAM) * scale


def test_gelu_pins():
    assert oracle.gelu(0.0) == 0.0
    for z in np.linspace(-6, 6, 121):
        exact = 0.5 * z * (1 + math.erf(z / math.sqrt(2)))
        assert abs(oracle.gelu(z) - exact) < 1e-3        # tanh form tracks the erf form closely
        e = 1e-6
        fd = (oracle.gelu(z + e) - oracle.gelu(z - e)) / (2 * e)
        assert abs(fd - oracle.gelu_grad(z)) < 1e-8
    assert oracle.gelu(20.0) == pytest.approx(20.0) and abs(oracle.gelu(-20.0)) < 1e-12


def test_forward_matches_layerwise_numpy():
    w = _params(0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((7, 216))
    y = oracle.mlp_forward(w, x)
    o = 0
    W1 = w[o:o + 128 * 216].reshape(128, 216); o += 128 * 216
    b1 = w[o:o + 128]; o += 128
    W2 = w[o:o + 128 * 128].reshape(128, 128); o += 128 * 128
    b2 = w[o:o + 128]; o += 128
    W3 = w[o:o + 4 * 128].reshape(4, 128); o += 4 * 128
    b3 = w[o:o + 4]; o += 4
    assert o == oracle.N_PARAM

    def gelu(z):
        return 0.5 * z * (1 + np.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))

    ref = gelu(gelu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    w = _params(2)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 216))
    dy = rng.standard_normal((3, 4))
    g = oracle.mlp_backward(w, x, dy)
    pick = np.concatenate([rng.choice(128 * 216, 40, replace=False),
                           27648 + rng.choice(128, 10, replace=False),
                           27776 + rng.choice(16384, 40, replace=False),
                           44160 + rng.choice(128, 10, replace=False),
                           44288 + rng.choice(512, 20, replace=False),
                           44800 + np.arange(4)])
    for i in pick:
        e = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[i] += e
        wm[i] -= e
        fd = ((oracle.mlp_forward(wp, x) * dy).sum() - (oracle.mlp_forward(wm, x) * dy).sum()) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    w0 = w.copy()
    oracle.adam(w, g, m, v, 1, 1e-3, eps=0.0)
    # bias correction makes the first step exactly lr * sign(g)
    assert np.allclose(w0 - w, 1e-3 * np.sign(g), rtol=1e-12, atol=0)
    # second step with the same gradient keeps the same step size
    oracle.adam(w, g, m, v, 2, 1e-3, eps=0.0)
    assert np.allclose(w0 - w, 2e-3 * np.sign(g), rtol=1e-12, atol=0)
