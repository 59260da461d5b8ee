"""Pins of the oracle's multi-resolution layer (Sec. 7, Sec. 7.1 step 1):
distances are evaluated only under the coarse layer's core cells, and for a
signed distance function the refined layer is the layer a dense sampling at
doubled resolution gives; for a field that is not a distance (steeper than
one) it is not, which shows the comparison can fail."""
import numpy as np
import pytest

import oracle
import synth


def _layers(shape, M, scale=1.0):
    d = synth.coarse_sdf(shape, M) * np.float32(scale)
    t = oracle.build_tables(M, d)
    core = np.nonzero(t.cell_type == 1)[0]
    child = synth.child_sdf(shape, core, M) * np.float32(scale)
    return d, child


SHAPES = [
    ("sphere", synth.sphere((0.5, 0.5, 0.5), 0.3), 16),
    ("off-centre sphere", synth.sphere((0.41, 0.55, 0.47), 0.27), 16),
    ("box", synth.box((0.5, 0.45, 0.52), (0.3, 0.2, 0.25)), 16),
    ("union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 16),
    ("shell", synth.shell((0.5, 0.5, 0.5), 0.3, 0.34), 32),
]


@pytest.mark.parametrize("name,shape,M", SHAPES, ids=[s[0] for s in SHAPES])
def test_refined_layer_equals_dense_sampling(name, shape, M):
    d, child = _layers(shape, M)
    ref, _ = oracle.refine_tables(M, d, child)
    dense = oracle.build_tables(2 * M, synth.coarse_sdf(shape, 2 * M))
    assert ref.n_packages == dense.n_packages > 0
    for a in ("cell_type", "cell_pkg", "pkg_cell", "pkg_type", "nbr"):
        assert np.array_equal(getattr(ref, a), getattr(dense, a)), a


def test_refined_core_lies_under_coarse_core():
    shape = synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))])
    M = 16
    d, child = _layers(shape, M, scale=4.0)
    ref, _ = oracle.refine_tables(M, d, child)
    coarse = oracle.build_tables(M, d)
    Mf = 2 * M
    f = np.nonzero(ref.cell_type == 1)[0]
    parent = (f % Mf) // 2 + M * (((f // Mf) % Mf) // 2 + M * ((f // (Mf * Mf)) // 2))
    assert f.size > 0 and np.all(coarse.cell_type[parent] == 1)
    # a field four times steeper than a distance: the coarse core misses fine
    # core cells of the dense sampling, so the two layers differ
    dense = oracle.build_tables(Mf, synth.coarse_sdf(shape, Mf) * np.float32(4.0))
    assert ref.n_packages < dense.n_packages
    assert set(f.tolist()) < set(np.nonzero(dense.cell_type == 1)[0].tolist())


def test_refined_far_field_sign_from_parent():
    # cells away from every coarse core cell are never evaluated: their
    # far-field side is their parent's
    shape = synth.sphere((0.5, 0.5, 0.5), 0.3)
    M = 16
    d, child = _layers(shape, M)
    ref, _ = oracle.refine_tables(M, d, child)
    Mf = 2 * M
    f = np.arange(Mf ** 3)
    parent = (f % Mf) // 2 + M * (((f // Mf) % Mf) // 2 + M * ((f // (Mf * Mf)) // 2))
    inactive = ref.cell_pkg < 2
    assert np.all(ref.cell_pkg[inactive] == (d[parent[inactive]] >= 0).astype(np.uint32))
    assert (ref.cell_pkg == 0).sum() > 0 and (ref.cell_pkg == 1).sum() > 0


def test_child_distances_are_the_dense_samples():
    shape = synth.box((0.5, 0.45, 0.52), (0.3, 0.2, 0.25))
    M = 8
    parents = np.array([0, 5, 77, M ** 3 - 1])
    child = synth.child_sdf(shape, parents, M)
    dense = synth.coarse_sdf(shape, 2 * M)
    Mf = 2 * M
    for r, c in enumerate(parents):
        i, j, k = c % M, (c // M) % M, c // (M * M)
        for b in range(8):
            fi, fj, fk = 2 * i + (b & 1), 2 * j + ((b >> 1) & 1), 2 * k + ((b >> 2) & 1)
            assert child[r, b] == dense[fi + Mf * (fj + Mf * fk)]
