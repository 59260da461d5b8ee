"""Leaky distances for the sign-correction tests: a signed distance with its
sign flipped inside random boxes, only at cells at least two cell sizes from
the surface (a broken inside/outside test away from the surface)."""
import numpy as np


def leaky(d, M, seed, n_boxes=6):
    """d with the sign flipped inside random boxes, only at cells at least two
    cell sizes from the surface (the near-surface signs stay right)."""
    rng = np.random.default_rng(seed)
    g = d.reshape(M, M, M).copy()      # [z, y, x]
    far = np.abs(g) >= 2.0 / M
    for _ in range(n_boxes):
        lo = rng.integers(0, M - 4, 3)
        hi = lo + rng.integers(2, max(3, M // 3), 3)
        box = np.zeros_like(far)
        box[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
        g[box & far] = -g[box & far]
    return g.ravel()
