"""Batched reinitialisation (GPU): every grid of a batch must come out bit
for bit equal to its own single-grid sweep, with and without graph replay,
for every kernel configuration; the single-grid sweep is checked against the
oracle elsewhere."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    sg.set_sweep_config(0, 1)
    return sg


@pytest.fixture(scope="module")
def bw(sg):
    from paper_2512_11473_amd import workload
    specs = synth.batch_shapes(7, 21, resolutions=(32, 64, 128))
    return workload.setup_batch(specs, 0.1)


def _singles(sg, bw, n_iter):
    out = []
    for p in bw.parts:
        p.reset()
        sg.reinitialize(p.grid, p.phi, p.scratch, n_iter)
        out.append(p.phi.clone())
    return out


@pytest.mark.parametrize("n_iter", [1, 6, 7])
def test_batch_equals_single_grids(sg, bw, n_iter):
    ref = _singles(sg, bw, n_iter)
    for variant, bpc in [(0, 1), (0, 4), (0, 0), (1, 2), (1, 8), (1, 0)]:
        bw.batch.set_config(variant, bpc)
        for use_graph in (False, True):
            bw.reset()
            bw.batch.reinitialize(bw.phi, bw.scratch, n_iter, use_graph=use_graph)
            torch.cuda.synchronize()
            for k, r in enumerate(ref):
                assert torch.equal(bw.slice(k, bw.phi), r), (variant, bpc, use_graph, k)


def test_graph_replays_match_eager(sg, bw):
    bw.batch.set_config(0, 4)
    bw.reset()
    bw.batch.reinitialize(bw.phi, bw.scratch, 10, use_graph=False)
    eager = bw.phi.clone()
    for rep in range(3):
        bw.reset()
        torch.cuda.synchronize()
        bw.batch.reinitialize(bw.phi, bw.scratch, 10, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(bw.phi, eager), rep
        # unrelated eager work between replays
        bw.scratch.mul_(0.5)
        torch.cuda.synchronize()


def test_autotune_keeps_results(sg, bw):
    v, b, table = bw.batch.autotune(bw.phi0, bw.scratch, reps=3)
    assert v in (0, 1) and b in (1, 2, 4, 8, 16, 0)
    assert table.shape == (2, 6)
    assert np.all(table > 0)
    ref = _singles(sg, bw, 4)
    bw.reset()
    bw.batch.reinitialize(bw.phi, bw.scratch, 4)
    for k, r in enumerate(ref):
        assert torch.equal(bw.slice(k, bw.phi), r)


def test_batch_member_against_oracle(sg, bw):
    # one member of the batch against the oracle, through the batched path
    k = int(np.argmin([p.grid.n_packages for p in bw.parts]))
    p = bw.parts[k]
    spec = synth.batch_shapes(7, 21, resolutions=(32, 64, 128))[k]
    bw.reset()
    bw.batch.reinitialize(bw.phi, bw.scratch, 12)
    run = oracle.setup(spec["shape"], spec["N"], 0.1, spec["noise_seed"])
    oracle.run_plain(run, 12)
    got = bw.slice(k, bw.phi)[2:].double().cpu().numpy().ravel()
    assert np.max(np.abs(got - run.phi[p.points.ravel()])) <= 1e-5 * run.h
