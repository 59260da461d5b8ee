"""Writes p8_integrals.json: the oracle's near-surface integrals of half-spaces
bounded by an axis-aligned plane (the kernel integral that Sec. 8 names, in
the reading of a dual-cell query point, Wendland C2 kernel with smoothing
length h and support 2h, exact plane-cube cut fractions).

For phi = x - (q_x + d h) the central differences are exactly (1, 0, 0), so
every cut fraction is the ramp clamp(1/2 + phi_j / h, 0, 1) and the integral
is a finite sum over the 32 support points.  Calls only the oracle.

    python tests/golden/make_p8_integrals.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

N = 16
H = 1.0 / N
D_OVER_H = (0.0, 0.25, 0.5, -0.25, -0.5, 0.9)


def main():
    i = np.arange(N ** 3)
    x = (np.stack([i % N, (i // N) % N, i // (N * N)], axis=1) + 0.5) * H
    p = 7 + N * (7 + N * 7)                     # an interior data point
    qx = x[p, 0] + 0.5 * H                      # its dual-cell query point
    rows = []
    for d in D_OVER_H:
        phi = x[:, 0] - (qx + d * H)
        out = oracle.integrals(N, H, 16 * H, phi, np.array([p], dtype=np.int64))[0]
        rows.append({"d_over_h": d, "K_W": float(out[0]), "hK_grad": [float(v) for v in out[1:]]})
    full = oracle.integrals(N, H, 16 * H, np.full(N ** 3, 5 * H), np.array([p], dtype=np.int64))[0]
    doc = {
        "what": "oracle integrals (K_W, h K_grad) at the dual-cell query of an interior point for the half-space "
                "phi = x - (q_x + d h); C = K_W of a support wholly on the phi > 0 side",
        "source": "tests/golden/make_p8_integrals.py (oracle only)",
        "N": N, "C": float(full[0]), "rows": rows,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "p8_integrals.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
