"""Per-element error scales of the surrogate kernels against the FP64 oracle.

The kernels evaluate the 216 -> 128 -> 128 -> 4 network with BF16 operands
and FP32 accumulation; the oracle evaluates it in FP64 on the same BF16
weight matrices (FP32 biases).  The difference is then made only of the
kernels' roundings.  A worst-case running error bound (every rounding at its
extreme and of one sign) overestimates it by about the square root of every
sum it passes through, about 100 times here, which would let a wrong entry
pass.  The scales below follow the probabilistic analysis of Higham and
Mary (SIAM J. Sci. Comput. 41, 2019): roundings are independent, mean-zero
errors, so their variances add through every sum and product.

- Rounding v to BF16 (8 significant bits) adds an error uniform over half an
  ulp, ulp <= 2 u |v| with u = 2^-8: variance <= u^2 v^2 / 3.  The same with
  w = 2^-24 for FP32.  A sum of K terms accumulated in FP32 adds at most K
  such FP32 errors of its partial sums.
- An error of variance s^2 in the argument of GELU or of its derivative
  passes with the squared derivative (first order); the tanh form's own FP32
  evaluation adds a few w relative to its terms.
- Through a matrix product the variances of the inputs are weighted by the
  squared entries.

Forward: z1 uses the input split into BF16 hi + lo parts (error of the lo
part, u^2 |x|); a1 = bf16(gelu(z1)), z2, a2 = bf16(gelu(z2)), y.  Backward
with a given dy: dA2 = dy W3 with the FP32 master W3 (the oracle has the BF16
one; that difference is computed exactly and counted in full), dZ2 =
bf16(dA2 gelu'(z2)), dA1 = dZ2 W2, dZ1 = bf16(dA1 gelu'(z1)); the weight
gradients contract BF16 operands over the batch: dW3 with bf16(dy) and a2,
dW2 with dZ2 and a1, dW1 with dZ1 and the BF16 hi part of x; the bias
gradients sum the BF16 dZ rows (db3 sums dy in FP32).

A test allows K_SIGMA standard deviations per element: over the 44,804
gradient entries of a test, a Gaussian would exceed that with probability
below 1e-6.
"""
from __future__ import annotations

import math

import numpy as np

U_BF16 = 2.0 ** -8
U_F32 = 2.0 ** -24
C_GELU = math.sqrt(2.0 / math.pi)

_SLICES = {"W1": (0, 27648), "b1": (27648, 27776), "W2": (27776, 44160), "b2": (44160, 44288),
           "W3": (44288, 44800), "b3": (44800, 44804)}


def _unpack(w):
    o = 0
    W1 = w[o:o + 128 * 216].reshape(128, 216); o += 128 * 216
    b1 = w[o:o + 128]; o += 128
    W2 = w[o:o + 128 * 128].reshape(128, 128); o += 128 * 128
    b2 = w[o:o + 128]; o += 128
    W3 = w[o:o + 4 * 128].reshape(4, 128); o += 4 * 128
    b3 = w[o:o + 4]
    return W1, b1, W2, b2, W3, b3


def _s(z):
    return 0.5 * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu(z):
    return z * _s(z)


def gelu_grad(z):
    s = _s(z)
    return s + 2.0 * z * s * (1.0 - s) * C_GELU * (1.0 + 3.0 * 0.044715 * z * z)


K_SIGMA = 6.0


def _v_bf16(v):
    return U_BF16 ** 2 * v * v / 3.0


def _v_acc(K, abs_sum):
    """Variance of the FP32 accumulation of K terms whose |terms| sum to abs_sum."""
    return K * (U_F32 * abs_sum) ** 2 / 3.0


def _gelu_dd(z):
    return (gelu_grad(z + 1e-5) - gelu_grad(z - 1e-5)) / 2e-5


def _v_gelu_eval(z):
    return (8 * U_F32 * z) ** 2 / 3.0


def _v_grad_eval(z):
    s = _s(z)
    t = np.abs(2.0 * z * s * (1.0 - s) * C_GELU * (1.0 + 3.0 * 0.044715 * z * z))
    return (16 * U_F32 * (s + t)) ** 2 / 3.0


def forward_scales(wq, x):
    """FP64 activations of the network with weights wq (BF16 matrices, FP32
    biases) and the variances of the kernels' errors in them."""
    W1, b1, W2, b2, W3, b3 = _unpack(wq)
    aW1, aW2, aW3 = np.abs(W1), np.abs(W2), np.abs(W3)
    z1 = x @ W1.T + b1
    v_z1 = (U_BF16 ** 4 / 3.0) * ((x * x) @ (W1 * W1).T) + _v_acc(450, np.abs(x) @ aW1.T + np.abs(b1))
    a1 = gelu(z1)
    v_a1 = gelu_grad(z1) ** 2 * v_z1 + _v_bf16(a1) + _v_gelu_eval(z1)
    z2 = a1 @ W2.T + b2
    v_z2 = v_a1 @ (W2 * W2).T + _v_acc(130, np.abs(a1) @ aW2.T + np.abs(b2))
    a2 = gelu(z2)
    v_a2 = gelu_grad(z2) ** 2 * v_z2 + _v_bf16(a2) + _v_gelu_eval(z2)
    y = a2 @ W3.T + b3
    v_y = v_a2 @ (W3 * W3).T + _v_acc(130, np.abs(a2) @ aW3.T + np.abs(b3))
    return dict(z1=z1, v_z1=v_z1, a1=a1, v_a1=v_a1, z2=z2, v_z2=v_z2, a2=a2, v_a2=v_a2, y=y, v_y=v_y)


def backward_scales(wq, w_master, x, dy):
    """Standard deviation [44804] of (kernel gradient - FP64 gradient on wq)
    for the loss sum_b dy_b . y_b, per parameter."""
    f = forward_scales(wq, x)
    _, _, W2, _, W3, _ = _unpack(wq)
    W3m = _unpack(w_master)[4]
    B = x.shape[0]
    dA2 = dy @ W3
    v_dA2 = (dy @ (W3m - W3)) ** 2 + _v_acc(4, np.abs(dy) @ np.abs(W3))
    g2, h2 = gelu_grad(f["z2"]), _gelu_dd(f["z2"])
    dZ2 = dA2 * g2
    v_dZ2 = g2 ** 2 * v_dA2 + dA2 ** 2 * (h2 ** 2 * f["v_z2"] + _v_grad_eval(f["z2"])) + _v_bf16(dZ2)
    dA1 = dZ2 @ W2
    v_dA1 = v_dZ2 @ (W2 * W2) + _v_acc(130, np.abs(dZ2) @ np.abs(W2))
    g1, h1 = gelu_grad(f["z1"]), _gelu_dd(f["z1"])
    dZ1 = dA1 * g1
    v_dZ1 = g1 ** 2 * v_dA1 + dA1 ** 2 * (h1 ** 2 * f["v_z1"] + _v_grad_eval(f["z1"])) + _v_bf16(dZ1)
    a1, a2 = f["a1"], f["a2"]
    x2, a12, a22 = x * x, a1 * a1, a2 * a2
    acc = B + 64                     # partial sums over 64-row workgroups, then over workgroups
    var = np.empty(44804)
    var[slice(*_SLICES["W1"])] = (v_dZ1.T @ x2 + (dZ1 * dZ1).T @ _v_bf16(x)
                                  + _v_acc(acc, np.abs(dZ1).T @ np.abs(x))).ravel()
    var[slice(*_SLICES["b1"])] = v_dZ1.sum(0) + _v_acc(acc, np.abs(dZ1).sum(0))
    var[slice(*_SLICES["W2"])] = (v_dZ2.T @ a12 + (dZ2 * dZ2).T @ f["v_a1"]
                                  + _v_acc(acc, np.abs(dZ2).T @ np.abs(a1))).ravel()
    var[slice(*_SLICES["b2"])] = v_dZ2.sum(0) + _v_acc(acc, np.abs(dZ2).sum(0))
    var[slice(*_SLICES["W3"])] = (_v_bf16(dy).T @ a22 + (dy * dy).T @ f["v_a2"]
                                  + _v_acc(acc, np.abs(dy).T @ np.abs(a2))).ravel()
    var[slice(*_SLICES["b3"])] = _v_acc(acc, np.abs(dy).sum(0))
    return np.sqrt(var)


def nonplanarity_f64(x):
    """Mean squared residual of each 6^3 window (rows of x, offsets x
    fastest) after its least-squares affine fit, by an explicit solve."""
    o = np.arange(6, dtype=np.float64)
    oz, oy, ox = np.meshgrid(o, o, o, indexing="ij")
    A = np.stack([np.ones(216), ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
    coef, *_ = np.linalg.lstsq(A, x.T, rcond=None)
    r = x.T - A @ coef
    return (r * r).mean(axis=0)


def nonplanarity_f32_bound(x):
    """Bound of the FP32 evaluation error of the kernel's non-planarity: the
    fit's coefficients c0 = s0 / 216 and c_a = s_a / 630 from moments summed
    per window row (six values: the row sum and its x moment, at most five
    roundings each) and then over 18 rows per lane, two lanes combined (at
    most 25 roundings in a chain, so within the 110 used below), then the
    explicit sum of squared residuals r_i = v_i - (c0 + c . o_i) in a second
    pass.

    With p~_i the plane through the computed coefficients, the computed sum
    is sum (r_i + e_i)^2 up to the rounding of the sum, where e_i is the
    plane's coefficient error at i (in the affine span, so sum r_i e_i = 0
    exactly) plus the rounding of three fused steps of the plane's value and
    of the subtraction.  Worst-case bounds: |ds0| <= 110 u sum |v|,
    |ds_a| <= 110 u sum |o_a v|, each division one more rounding."""
    o = np.arange(6, dtype=np.float64) - 2.5
    oz, oy, ox = np.meshgrid(o, o, o, indexing="ij")
    offs = [c.ravel() for c in (ox, oy, oz)]
    u = U_F32
    ax = np.abs(x)
    c0 = x.mean(1)
    cs = [(x * c).sum(1) / 630.0 for c in offs]
    plane = c0[:, None] + sum(c[:, None] * oc[None, :] for c, oc in zip(cs, offs))
    r = x - plane
    d0 = 110 * u * ax.sum(1) / 216.0 + u * np.abs(c0)
    ds = [110 * u * (ax * np.abs(oc)).sum(1) / 630.0 + u * np.abs(c) for c, oc in zip(cs, offs)]
    dp = d0[:, None] + sum(d[:, None] * np.abs(oc)[None, :] for d, oc in zip(ds, offs))
    amp = np.abs(c0)[:, None] + sum(np.abs(c)[:, None] * np.abs(oc)[None, :] for c, oc in zip(cs, offs))
    ev = 3 * u * (amp + dp) + u * (np.abs(r) + dp + 3 * u * (amp + dp))
    E = dp + ev
    tot = 2 * (np.abs(r) * ev).sum(1) + (E * E).sum(1) + 110 * u * ((np.abs(r) + E) ** 2).sum(1)
    return tot / 216.0 * (1 + 1e-6)
