"""Stored values of the near-surface integral (the kernel integral of Sec. 8
in the reading of a dual-cell query, Wendland C2 kernel, support 2h and
exact plane-cube cut fractions) for half-spaces bounded by an axis-aligned
plane, pinned two ways:

- against values of the same reading computed independently, before the
  oracle was written, and quoted here to the digits they were given in
  (16 for K_W and C, 9 for h K_grad);
- the file itself, written by tests/golden/make_p8_integrals.py from the
  oracle, must stay reproducible: a later change to the oracle's arithmetic
  that moves any value by more than 1e-12 fails here.
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "p8_integrals.json")

# d / h -> (K_W, h K_grad x), independent evaluation of the reading
INDEPENDENT = {
    0.0: (0.49027270736178424, 0.865663036),
    0.25: (0.3692408822561619, 0.664871858),
    0.5: (0.24820905715053962, 0.464080680),
    -0.25: (0.6113045324674066, 0.664871858),
}
C_INDEPENDENT = 0.9805454147235685


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_agrees_with_independent_values(golden):
    assert golden["C"] == pytest.approx(C_INDEPENDENT, abs=1e-12)
    rows = {r["d_over_h"]: r for r in golden["rows"]}
    for d, (kw, gx) in INDEPENDENT.items():
        assert rows[d]["K_W"] == pytest.approx(kw, abs=1e-12), d
        assert rows[d]["hK_grad"][0] == pytest.approx(gx, abs=5e-10), d
        assert abs(rows[d]["hK_grad"][1]) < 1e-12 and abs(rows[d]["hK_grad"][2]) < 1e-12
    # d = 0: the plane through the query point splits the support evenly
    assert rows[0.0]["K_W"] == pytest.approx(golden["C"] / 2, abs=1e-12)
    # d -> -d: the complement, K_W -> C - K_W, the gradient unchanged
    for d in (0.25, 0.5):
        assert rows[d]["K_W"] + rows[-d]["K_W"] == pytest.approx(golden["C"], abs=1e-12)
        assert rows[d]["hK_grad"][0] == pytest.approx(rows[-d]["hK_grad"][0], abs=1e-12)


def test_oracle_reproduces_golden(golden):
    N = golden["N"]
    H = 1.0 / N
    i = np.arange(N ** 3)
    x = (np.stack([i % N, (i // N) % N, i // (N * N)], axis=1) + 0.5) * H
    p = 7 + N * (7 + N * 7)
    qx = x[p, 0] + 0.5 * H
    for r in golden["rows"]:
        phi = x[:, 0] - (qx + r["d_over_h"] * H)
        out = oracle.integrals(N, H, 16 * H, phi, np.array([p], dtype=np.int64))[0]
        assert out[0] == pytest.approx(r["K_W"], abs=1e-12)
        assert np.allclose(out[1:], r["hK_grad"], atol=1e-12, rtol=0)
    assert oracle.c_full() == pytest.approx(golden["C"], abs=1e-12)
