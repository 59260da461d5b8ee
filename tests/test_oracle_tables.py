"""Pins of the oracle's package tables against independent constructions.

Activation (Sec. 7.1 steps 1-2), numbering (Sec. 5, Sec. 7.1 step 3),
neighbour table (Sec. 5.2, Sec. 7.1 step 5) and the index shift of Sec. 5.2.
Each expected value comes from a library routine (scipy dilation, numpy
ordering, numpy padding) or from exhaustive enumeration, never from the
oracle's own loops.
"""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth


def _core_dilation(core):
    """Inner = 26-neighbourhood dilation of core minus core (scipy)."""
    st = np.ones((3, 3, 3), dtype=bool)
    dil = ndimage.binary_dilation(core, structure=st)
    return dil & ~core


def _expected_types(M, d, lc):
    d3 = d.reshape(M, M, M)  # [z][y][x]
    core = np.abs(d3.astype(np.float64)) < lc
    inner = _core_dilation(core)
    t = np.zeros((M, M, M), dtype=np.uint8)
    t[core] = 1
    t[inner] = 2
    return t.ravel()


def test_index_shift_exhaustive():
    # Sec. 5.2: shift s in [-4, 7] addresses the 3 neighbour slots of one axis.
    for s in range(-4, 8):
        slot, data = oracle.index_shift(s)
        assert slot == s // 4 + 1          # floor division: which package along the axis
        assert data == s % 4               # position inside it
        assert 0 <= slot <= 2 and 0 <= data <= 3
    # 3D: every shift in [-4,7]^3 lands on a distinct (slot, data) pair
    seen = set()
    for s in itertools.product(range(-4, 8), repeat=3):
        key = tuple(oracle.index_shift(c) for c in s)
        seen.add(key)
    assert len(seen) == 12 ** 3


def test_activation_all_core_patterns_m2():
    # All 256 core patterns on a 2x2x2 coarse grid; every cell neighbours every other.
    M, lc = 2, 0.5
    rng = np.random.default_rng(0)
    for pattern in range(256):
        core = np.array([(pattern >> c) & 1 for c in range(8)], dtype=bool)
        d = np.where(core, rng.uniform(-0.49, 0.49, 8), rng.choice([-1, 1], 8) * rng.uniform(0.5, 2, 8))
        d = d.astype(np.float32)
        got = oracle.classify(M, lc, d)
        assert np.array_equal(got, _expected_types(M, d, lc)), pattern


@pytest.mark.parametrize("M", [1, 3, 4, 5, 8])
def test_activation_random_with_ties(M):
    lc = 1.0 / M
    rng = np.random.default_rng(M)
    choices = np.array([lc, -lc, 0.0, -0.0, 0.5 * lc, -0.5 * lc, 2 * lc, -2 * lc, 1.5 * lc], dtype=np.float32)
    for trial in range(20):
        d = rng.choice(choices, M ** 3).astype(np.float32)
        if trial % 2:
            d = (d + rng.uniform(-0.01, 0.01, M ** 3).astype(np.float32) * (rng.uniform(size=M ** 3) < 0.3))
            d = d.astype(np.float32)
        got = oracle.classify(M, lc, d)
        assert np.array_equal(got, _expected_types(M, d, lc))


def _check_tables(tab: oracle.Tables, d: np.ndarray):
    M = tab.M
    n = M ** 3
    active = np.nonzero(tab.cell_type)[0]
    P = active.shape[0]
    assert tab.n_packages == P
    # ids 2.. in ascending linear order (numpy's own ordering of nonzero)
    assert np.array_equal(tab.cell_pkg[active], np.arange(2, P + 2, dtype=np.uint32))
    assert np.array_equal(tab.pkg_cell[2:], active.astype(np.uint32))
    assert np.array_equal(tab.pkg_type[2:], tab.cell_type[active])
    assert tab.pkg_cell[0] == 0xFFFFFFFF and tab.pkg_cell[1] == 0xFFFFFFFF
    assert tab.pkg_type[0] == 0 and tab.pkg_type[1] == 0
    # far field by sign (negative -> 0, zero / -0.0 / positive -> 1)
    inactive = np.ones(n, dtype=bool)
    inactive[active] = False
    exp_far = np.where(d[inactive] < 0, 0, 1).astype(np.uint32)
    assert np.array_equal(tab.cell_pkg[inactive], exp_far)
    # neighbour table from a padded copy of the map (padding = positive far field)
    cp = np.pad(tab.cell_pkg.reshape(M, M, M), 1, constant_values=1)
    for s in range(27):
        dx, dy, dz = s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1
        shifted = cp[1 + dz:1 + dz + M, 1 + dy:1 + dy + M, 1 + dx:1 + dx + M].ravel()
        assert np.array_equal(tab.nbr[2:, s], shifted[active]), s
    assert np.all(tab.nbr[0] == 0) and np.all(tab.nbr[1] == 1)
    assert np.array_equal(tab.nbr[:, 13], np.arange(P + 2, dtype=np.uint32))
    # every in-domain 26-neighbour of a core package is activated
    inside = np.pad(np.ones((M, M, M), dtype=bool), 1, constant_values=False)
    is_core = tab.pkg_type[2:] == 1
    for s in range(27):
        dx, dy, dz = s % 3 - 1, (s // 3) % 3 - 1, s // 9 - 1
        ins = inside[1 + dz:1 + dz + M, 1 + dy:1 + dy + M, 1 + dx:1 + dx + M].ravel()[active]
        assert np.all(tab.nbr[2:, s][is_core & ins] >= 2)


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8])
def test_tables_random_tiny(M):
    rng = np.random.default_rng(100 + M)
    lc = 1.0 / M
    for _ in range(10):
        d = (rng.uniform(-3, 3, M ** 3) * lc).astype(np.float32)
        d[rng.uniform(size=M ** 3) < 0.1] = np.float32(lc)
        d[rng.uniform(size=M ** 3) < 0.05] = np.float32(-0.0)
        tab = oracle.build_tables(M, d)
        _check_tables(tab, d)


def test_tables_sphere64_counts():
    # Sphere r = 0.3 at 64^3 data points (16^3 coarse cells).
    cfg = synth.config_c1()
    d = synth.coarse_sdf(cfg["shape"], 16)
    tab = oracle.build_tables(16, d)
    _check_tables(tab, d)
    assert int((tab.pkg_type == 1).sum()) == 632
    assert tab.n_packages == 1632


def test_tables_prism512_counts():
    # Extruded triangular prism at 512^3 data points (128^3 coarse cells).
    cfg = synth.config_c2()
    d = synth.coarse_sdf(cfg["shape"], 128)
    tab = oracle.build_tables(128, d)
    _check_tables(tab, d)
    assert int((tab.pkg_type == 1).sum()) == 56880
    assert tab.n_packages == 124308
