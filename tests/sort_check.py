"""Host-side checks of the particle sort: the keys recomputed from the
positions in the kernel's FP32 arithmetic, and the one order a stable sort
by them can give."""
import numpy as np


def _spread3(v):
    """Bit b of v to bit 3b (Morton interleave)."""
    out = np.zeros_like(v)
    for b in range(10):
        out |= ((v >> b) & 1) << (3 * b)
    return out


def host_keys(M, pos, h):
    """Sort key of every particle: the Morton code (x in the lowest bit) of its
    home coarse cell clamp(floor(x * (1/h) * 0.25), 0, M - 1) per axis, all
    in FP32 as on the device, NaN clamping to 0."""
    inv_h = np.float32(1.0 / h)
    u = pos.astype(np.float32) * inv_h
    c = np.fmin(np.fmax(np.floor(u * np.float32(0.25)), np.float32(0)), np.float32(M - 1)).astype(np.int64)
    return _spread3(c[:, 0]) | (_spread3(c[:, 1]) << 1) | (_spread3(c[:, 2]) << 2)


def assert_sorted(M, h, pos, pos_sorted, perm):
    """The sort is stable, so its permutation is unique: the stable argsort of
    the host keys; pos_sorted = pos[perm] bit for bit."""
    keys = host_keys(M, pos, h)
    want = np.argsort(keys, kind="stable")
    assert np.array_equal(perm.astype(np.int64), want)
    assert np.array_equal(pos_sorted.view(np.uint32), pos[want].view(np.uint32))
    return keys[want]
