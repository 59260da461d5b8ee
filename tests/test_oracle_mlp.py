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


def test_adam_five_steps_against_the_unrolled_moments():
    # Kingma & Ba (2015, Sec. 3) write the moments as exponentially weighted
    # sums, m_t = (1 - b1) sum_i b1^(t-i) g_i and v_t = (1 - b2) sum_i
    # b2^(t-i) g_i^2, bias-corrected by 1 - b^t; the update divides by
    # sqrt(v_hat) + eps.  The oracle runs the recursion; here the sums are
    # formed from the whole gradient history at every step, with gradients
    # that change sign and scale, and an eps large enough to tell where it
    # enters.
    rng = np.random.default_rng(9)
    n, steps, lr, b1, b2, eps = 500, 5, 3e-3, 0.8, 0.95, 1e-2
    w = rng.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    gs = [rng.standard_normal(n) * rng.uniform(0.05, 3.0, n) for _ in range(steps)]
    w_ref = w.copy()
    for t in range(1, steps + 1):
        oracle.adam(w, gs[t - 1], m, v, t, lr, beta1=b1, beta2=b2, eps=eps)
        G = np.array(gs[:t])
        k = np.arange(t - 1, -1, -1)[:, None]           # t - i for i = 1..t
        m_sum = (1 - b1) * (b1 ** k * G).sum(axis=0)
        v_sum = (1 - b2) * (b2 ** k * G * G).sum(axis=0)
        # rounding of the two summation orders, relative to the sum of |terms|
        assert np.all(np.abs(m - m_sum) <= 1e-14 * (1 - b1) * (b1 ** k * np.abs(G)).sum(axis=0))
        assert np.allclose(v, v_sum, rtol=1e-13, atol=0)
        w_ref -= lr * (m_sum / (1 - b1 ** t)) / (np.sqrt(v_sum / (1 - b2 ** t)) + eps)
        assert np.allclose(w, w_ref, rtol=1e-13, atol=1e-16)


def test_adam_scale_invariance_and_antisymmetry():
    # With eps = 0 the update is invariant under g -> c g (c > 0) and flips
    # sign under g -> -g, at every step of a varying-gradient sequence.
    rng = np.random.default_rng(10)
    n = 300
    gs = [rng.standard_normal(n) for _ in range(4)]
    w0 = rng.standard_normal(n)
    runs = {}
    for name, c in (("base", 1.0), ("scaled", 37.5), ("negated", -1.0)):
        w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
        for t, g in enumerate(gs, start=1):
            oracle.adam(w, c * g, m, v, t, 1e-3, eps=0.0)
        runs[name] = w - w0
    assert np.allclose(runs["scaled"], runs["base"], rtol=1e-12, atol=1e-18)
    assert np.allclose(runs["negated"], -runs["base"], rtol=1e-12, atol=1e-18)
    # a constant gradient keeps a step of exactly lr per step
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        oracle.adam(w, gs[0], m, v, t, 1e-3, eps=0.0)
    assert np.allclose(w0 - w, 5e-3 * np.sign(gs[0]), rtol=1e-12, atol=0)
