"""Pins of the oracle's sign correction by diffusion (Sec. 7.2, the coarse
step on the mesh cells): a distance function is left unchanged; signs flipped
in regions away from the surface (a leaky inside/outside test) are restored;
the result agrees with an independent labelling of the connected regions of
uncertain cells; the number of rounds is the diffusion distance."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from leaky import leaky as _leaky


SHAPES = [
    ("sphere", synth.sphere((0.5, 0.5, 0.5), 0.3), 24),
    ("union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 32),
    ("shell", synth.shell((0.5, 0.5, 0.5), 0.25, 0.32), 32),
]


@pytest.mark.parametrize("name,shape,M", SHAPES, ids=[s[0] for s in SHAPES])
def test_distance_function_unchanged(name, shape, M):
    d = synth.coarse_sdf(shape, M)
    out, rounds = oracle.correct_signs(M, d)
    assert np.array_equal(out.view(np.uint32), d.view(np.uint32))
    assert rounds > 0


@pytest.mark.parametrize("name,shape,M", SHAPES, ids=[s[0] for s in SHAPES])
def test_leaks_are_repaired(name, shape, M):
    d = synth.coarse_sdf(shape, M)
    for seed in range(3):
        bad = _leaky(d, M, seed)
        assert np.sum(np.sign(bad) != np.sign(d)) > 20
        out, _ = oracle.correct_signs(M, bad)
        assert np.array_equal(out, d)
        assert np.array_equal(oracle.build_tables(M, out).cell_pkg, oracle.build_tables(M, d).cell_pkg)


def test_agrees_with_region_labelling():
    # every 6-connected region of non-core cells takes the sign of the core
    # cells on its border (one sign per region for these inputs); regions that
    # touch no core cell keep their input signs
    M = 32
    shape = synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))])
    d = synth.coarse_sdf(shape, M)
    bad = _leaky(d, M, 11, n_boxes=10)
    out, _ = oracle.correct_signs(M, bad)
    g = bad.reshape(M, M, M)
    core = np.abs(g.astype(np.float64)) < 1.0 / M
    lab, n = ndimage.label(~core)
    pos_core = core & ~(g < 0)
    neg_core = core & (g < 0)
    want = g.copy()
    st = ndimage.generate_binary_structure(3, 1)
    for r in range(1, n + 1):
        reg = lab == r
        ring = ndimage.binary_dilation(reg, st) & ~reg
        p, q = (ring & pos_core).any(), (ring & neg_core).any()
        assert not (p and q)
        if p:
            want[reg] = np.abs(g[reg])
        elif q:
            want[reg] = -np.abs(g[reg])
    assert np.array_equal(out.reshape(M, M, M), want)


def test_rounds_are_the_diffusion_distance():
    # a single core cell in a corner of an otherwise uncertain grid: the sign
    # spreads one face step per round, so the far corner is reached after
    # 3 (M - 1) rounds, and every cell takes the core cell's sign
    M = 9
    d = np.full(M ** 3, 5.0, dtype=np.float32)
    d[0] = -0.01
    out, rounds = oracle.correct_signs(M, d)
    assert rounds == 3 * (M - 1)
    assert np.all(out[1:] == -5.0) and out[0] == d[0]
    # no core cell: nothing is decided, nothing changes
    e = np.where(np.arange(M ** 3) % 2 == 0, 3.0, -3.0).astype(np.float32)
    out, rounds = oracle.correct_signs(M, e)
    assert rounds == 0 and np.array_equal(out, e)


def test_positive_wins_a_tie():
    # an uncertain cell between a positive and a negative core cell
    M = 3
    d = np.full(M ** 3, 7.0, dtype=np.float32)
    d[0 + 3 * 1 + 9 * 1] = 0.1       # (0, 1, 1) positive core
    d[2 + 3 * 1 + 9 * 1] = -0.1      # (2, 1, 1) negative core
    out, _ = oracle.correct_signs(M, d, lc=0.5)
    assert out[1 + 3 * 1 + 9 * 1] == 7.0


# --------------------------------------------------------------------------
# The refined step on the data packages (Sec. 7.2): limited to the inner
# packages, whose points take their sign by diffusion from the core packages
# and the far field
# --------------------------------------------------------------------------

def _band_state(shape, N, amp=0.1, seed=3):
    run = oracle.setup(shape, N, amp, seed)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    return run, dense


def _leaky_points(run, dense, seed, n_boxes=6):
    """The inner packages' points with the sign flipped inside random boxes."""
    N = run.N
    rng = np.random.default_rng(seed)
    bad = dense.copy()
    inner = oracle.active_points(run.tab, pkg_types=(2,))
    i, j, k = inner % N, (inner // N) % N, inner // (N * N)
    for _ in range(n_boxes):
        lo = rng.integers(0, N - 8, 3)
        hi = lo + rng.integers(4, N // 3, 3)
        sel = (i >= lo[0]) & (i < hi[0]) & (j >= lo[1]) & (j < hi[1]) & (k >= lo[2]) & (k < hi[2])
        bad[inner[sel]] = -bad[inner[sel]]
    return bad


POINT_SHAPES = [
    ("sphere", synth.sphere((0.5, 0.5, 0.5), 0.3), 64),
    ("union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 64),
    ("shell", synth.shell((0.5, 0.5, 0.5), 0.25, 0.32), 128),
]


@pytest.mark.parametrize("name,shape,N", POINT_SHAPES, ids=[s[0] for s in POINT_SHAPES])
def test_point_signs_unchanged_and_repaired(name, shape, N):
    run, dense = _band_state(shape, N)
    out, rounds = oracle.correct_point_signs(run.N, run.tab, dense)
    assert np.array_equal(out, dense) and rounds > 0
    flipped = 0
    for seed in range(3):
        bad = _leaky_points(run, dense, seed)
        flipped += int(np.sum(bad != dense))
        out, _ = oracle.correct_point_signs(run.N, run.tab, bad)
        assert np.array_equal(out, dense)
    assert flipped > 1000


def test_point_signs_agree_with_region_labelling():
    run, dense = _band_state(POINT_SHAPES[1][1], 64)
    bad = _leaky_points(run, dense, 11, n_boxes=10)
    out, _ = oracle.correct_point_signs(run.N, run.tab, bad)
    N = run.N
    g = bad.reshape(N, N, N)
    uncertain = np.zeros(N ** 3, dtype=bool)
    uncertain[oracle.active_points(run.tab, pkg_types=(2,))] = True
    uncertain = uncertain.reshape(N, N, N)
    lab, n = ndimage.label(uncertain)
    decided = ~uncertain
    pos = decided & ~(g < 0)
    neg = decided & (g < 0)
    st = ndimage.generate_binary_structure(3, 1)
    want = g.copy()
    for r in range(1, n + 1):
        reg = lab == r
        ring = ndimage.binary_dilation(reg, st) & ~reg
        # a region touching a domain face sees the positive far field there
        face = reg[0].any() or reg[-1].any() or reg[:, 0].any() or reg[:, -1].any() or \
            reg[:, :, 0].any() or reg[:, :, -1].any()
        p, q = (ring & pos).any() or face, (ring & neg).any()
        assert not (p and q)
        if p:
            want[reg] = np.abs(g[reg])
        elif q:
            want[reg] = -np.abs(g[reg])
    assert np.array_equal(out.reshape(N, N, N), want)
