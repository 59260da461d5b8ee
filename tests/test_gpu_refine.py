"""The multi-resolution layer build (Sec. 7, Sec. 7.1 step 1) against the
oracle, bit for bit: one refinement of several shapes, a field steeper than a
distance (where the refined layer is not the dense one), a chain of three
refinements, and the torus at full size (2048^3 data points refined from the
1024^3 layer)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tables_check import assert_tables_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    return sg


def _np_tables(g):
    return {k: v.cpu().numpy() for k, v in g.tables().items()}


def _core_cells(g):
    t = g.tables()
    core = t["core_list"].cpu().numpy().astype(np.int64)
    return t["pkg_cell"].cpu().numpy().view(np.uint32)[core].astype(np.int64)


def _refine(sg, g, shape, M, scale=1.0):
    child = synth.child_sdf(shape, _core_cells(g), M) * np.float32(scale)
    return sg.build_packages_refined(g, torch.from_numpy(child).cuda()), child


CASES = [
    ("sphere", synth.sphere((0.5, 0.5, 0.5), 0.3), 16, 1.0),
    ("union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 16,
     1.0),
    ("shell", synth.shell((0.5, 0.5, 0.5), 0.3, 0.34), 32, 1.0),
    ("steep union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]),
     16, 4.0),
    ("off-grid sphere", synth.sphere((0.43, 0.52, 0.49), 0.31), 64, 1.0),
]


@pytest.mark.parametrize("name,shape,M,scale", CASES, ids=[c[0] for c in CASES])
def test_refined_build_matches_oracle(sg, name, shape, M, scale):
    d = synth.coarse_sdf(shape, M) * np.float32(scale)
    g0 = sg.build_packages(torch.from_numpy(d).cuda(), 1.0 / (4 * M))
    g1, child = _refine(sg, g0, shape, M, scale)
    ref, _ = oracle.refine_tables(M, d, child)
    assert g1.n_packages == ref.n_packages and g1.h == pytest.approx(1.0 / (8 * M), rel=0, abs=0)
    assert_tables_equal(_np_tables(g1), ref)
    dense = sg.build_packages(torch.from_numpy(synth.coarse_sdf(shape, 2 * M) * np.float32(scale)).cuda(),
                              1.0 / (8 * M))
    same = all(np.array_equal(a, b) for a, b in zip(_np_tables(g1).values(), _np_tables(dense).values()))
    assert same == (scale == 1.0)      # a distance function refines to its dense sampling; a steeper field does not


def test_refinement_chain(sg):
    shape = synth.union([synth.sphere((0.35, 0.45, 0.5), 0.2), synth.box((0.65, 0.55, 0.45), (0.15, 0.2, 0.18))])
    M = 8
    d = synth.coarse_sdf(shape, M)
    g = sg.build_packages(torch.from_numpy(d).cuda(), 1.0 / (4 * M))
    for level in range(3):
        g_next, child = _refine(sg, g, shape, M)
        ref, d = oracle.refine_tables(M, d, child)
        assert_tables_equal(_np_tables(g_next), ref)
        g.destroy()
        g, M = g_next, 2 * M
    assert M == 64 and g.n_packages > 10000


def test_refine_without_core(sg):
    # a band-free grid (everything far inside): no core cell, nothing to evaluate
    M = 8
    d = np.full(M ** 3, -1.0, dtype=np.float32)
    g0 = sg.build_packages(torch.from_numpy(d).cuda(), 1.0 / (4 * M))
    assert g0.n_core == 0
    g1 = sg.build_packages_refined(g0, None)
    t = _np_tables(g1)
    assert g1.n_packages == 0 and np.all(t["cell_pkg"].view(np.uint32) == 0)
    with pytest.raises(ValueError):
        g2 = sg.build_packages(torch.from_numpy(synth.coarse_sdf(synth.sphere((0.5, 0.5, 0.5), 0.3), M)).cuda(),
                               1.0 / (4 * M))
        sg.build_packages_refined(g2, torch.zeros(3, device="cuda"))


def test_torus2048_refined_from_1024(sg):
    cfg = synth.config_c5()
    shape = cfg["shape"]
    Mc = cfg["N"] // 8                      # 256: the 1024^3 layer
    d = synth.coarse_sdf(shape, Mc)
    g0 = sg.build_packages(torch.from_numpy(d).cuda(), 1.0 / (4 * Mc))
    child = synth.child_sdf(shape, _core_cells(g0), Mc)
    g1 = sg.build_packages_refined(g0, torch.from_numpy(child).cuda())
    ref, _ = oracle.refine_tables(Mc, d, child)
    assert g1.n_packages == ref.n_packages > 1_000_000
    assert_tables_equal(_np_tables(g1), ref)
