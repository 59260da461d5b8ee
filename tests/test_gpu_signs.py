"""Sign correction by diffusion on the GPU (Sec. 7.2, coarse step) against
the oracle, bit for bit, with the round count; in place and out of place; a
grid width that is not a multiple of 64; and the torus's 512^3 coarse grid at
full size, where the repaired distances must be the unbroken ones."""
import numpy as np
import pytest
import torch

import oracle
import synth
from leaky import leaky

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    return sg


CASES = [
    ("sphere", synth.sphere((0.5, 0.5, 0.5), 0.3), 24),
    ("union", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15), synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 72),
    ("shell", synth.shell((0.5, 0.5, 0.5), 0.25, 0.32), 128),
]


@pytest.mark.parametrize("name,shape,M", CASES, ids=[c[0] for c in CASES])
def test_sign_correction_matches_oracle(sg, name, shape, M):
    d = synth.coarse_sdf(shape, M)
    for seed in range(2):
        bad = leaky(d, M, seed, n_boxes=8)
        ref, ref_rounds = oracle.correct_signs(M, bad)
        x = torch.from_numpy(bad).cuda()
        out = torch.empty_like(x)
        rounds = sg.correct_signs(x, 1.0 / (4 * M), out)
        assert rounds == ref_rounds > 0
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        assert torch.equal(x, torch.from_numpy(bad).cuda())          # the input is only read
        rounds2 = sg.correct_signs(x, 1.0 / (4 * M))                 # in place
        assert rounds2 == ref_rounds and np.array_equal(x.cpu().numpy().view(np.uint32), ref.view(np.uint32))
        # the leaks are repaired (no face of these shapes passes through a row of
        # cell centres at this M, where a cell at exactly the core threshold
        # could border a core cell of the other sign)
        assert np.array_equal(ref, d)


def test_sign_correction_edge_cases(sg):
    # one core cell in a corner: the sign reaches the far corner after 3 (M - 1) rounds
    M = 9
    d = np.full(M ** 3, 5.0, dtype=np.float32)
    d[0] = -0.01
    x = torch.from_numpy(d).cuda()
    assert sg.correct_signs(x, 1.0 / (4 * M)) == 3 * (M - 1)
    assert np.all(x.cpu().numpy()[1:] == -5.0)
    # no core cell: nothing changes
    e = np.where(np.arange(M ** 3) % 2 == 0, 3.0, -3.0).astype(np.float32)
    y = torch.from_numpy(e).cuda()
    assert sg.correct_signs(y, 1.0 / (4 * M)) == 0 and np.array_equal(y.cpu().numpy(), e)
    with pytest.raises(ValueError):
        sg.correct_signs(torch.zeros(10, device="cuda"), 0.1)


def test_torus2048_coarse_grid_repaired(sg):
    # the torus of the 2048^3 workload without its displacement (an exact
    # distance function), on its 512^3 coarse grid
    cfg = synth.config_c5()
    M = cfg["N"] // 4
    d = synth.coarse_sdf(synth.torus((0.5, 0.5, 0.5), 0.35, 0.1), M)
    bad = leaky(d, M, 3, n_boxes=12)
    assert np.sum(np.sign(bad) != np.sign(d)) > 1_000_000
    x = torch.from_numpy(bad).cuda()
    rounds = sg.correct_signs(x, 1.0 / cfg["N"])
    assert rounds > 10
    assert np.array_equal(x.cpu().numpy(), d)


# the refined step on the data packages
def _leaky_points(run, dense, seed, n_boxes=6):
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


POINT_CASES = [
    ("sphere64", synth.sphere((0.5, 0.5, 0.5), 0.3), 64, torch.float32),
    ("union64-f64", synth.union([synth.sphere((0.3, 0.4, 0.5), 0.15),
                                 synth.box((0.62, 0.6, 0.5), (0.2, 0.15, 0.2))]), 64, torch.float64),
    ("shell128", synth.shell((0.5, 0.5, 0.5), 0.25, 0.32), 128, torch.float32),
]


@pytest.mark.parametrize("name,shape,N,dtype", POINT_CASES, ids=[c[0] for c in POINT_CASES])
def test_package_sign_correction_matches_oracle(sg, name, shape, N, dtype):
    from paper_2512_11473_amd import workload
    npd = np.float32 if dtype == torch.float32 else np.float64
    wl = workload.setup(shape, N, 0.1, 3, dtype=dtype)
    run = oracle.setup(shape, N, 0.1, 3, phi0_dtype=npd)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    pts = wl.points.ravel()
    for seed in range(2):
        bad = _leaky_points(run, dense, seed, n_boxes=8)
        ref, ref_rounds = oracle.correct_point_signs(run.N, run.tab, bad)
        phi = wl.phi.clone()
        phi[2:] = torch.from_numpy(bad[pts].reshape(-1, 64).astype(npd)).cuda()
        rounds = sg.correct_package_signs(wl.grid, phi)
        assert rounds == ref_rounds > 0
        got = phi[2:].double().cpu().numpy().ravel()
        assert np.array_equal(got, ref[pts])
        assert np.array_equal(ref, dense)                  # the leaks are repaired
        assert torch.equal(phi[:2], wl.phi[:2])            # far-field rows untouched
