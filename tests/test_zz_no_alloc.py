"""The allocation-free learned integrals against the allocating entry (GPU).

sgrid_compute_near_surface_integrals_noalloc runs the same kernels with the
fallback list in the library's fixed per-device array, in chunks of 32,768
core packages.  Two calls in a row, the second on a smaller grid, must give
the outputs and the fallback count of sgrid_compute_near_surface_integrals
with the same model, bit for bit: the first grid (the prism at 512^3,
56,880 core packages) spans two chunks, the second (the sphere at 64^3) one.
The gate threshold is the median non-planarity of the grid's windows, so
about half of the non-saturated points take the fallback.
"""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    return sg


def _grid(cfg, n_iter=5):
    import paper_2512_11473_amd as sg
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
    return wl


def _median_tau(sg, wl):
    from paper_2512_11473_amd import surrogate
    n = wl.grid.n_core * 64
    x = torch.empty((n, 216), device="cuda")
    un = torch.empty(n, dtype=torch.uint8, device="cuda")
    sg.gather_windows(wl.grid, wl.phi, x, un)
    res = surrogate.nonplanarity(x[un.bool()])
    return float(res.median())


def _compare(sg, model, wl, with_count=True):
    n = wl.grid.n_core * 64
    ref = torch.empty((4, n), device="cuda")
    got = torch.full((4, n), float("nan"), device="cuda")
    nf_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
    nf_got = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    sg.compute_near_surface_integrals(wl.grid, wl.phi, ref, model=model, n_fallback=nf_ref)
    sg.compute_near_surface_integrals_noalloc(wl.grid, wl.phi, got, model, nf_got if with_count else None)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    if with_count:
        assert int(nf_got.item()) == int(nf_ref.item())
    return int(nf_ref.item()), n


def test_noalloc_matches_allocating_entry(sg):
    from paper_2512_11473_amd import surrogate
    model = sg.Mlp(surrogate.init_params(3, 2.0))
    big = _grid(synth.config_c2())
    assert big.grid.n_core > 32768                     # two chunks
    model.set_gate(_median_tau(sg, big))
    print(f"prism512: {big.grid.n_core} core packages", flush=True)
    nf, n = _compare(sg, model, big)
    assert nf > 0.05 * n                               # the fallback path is exercised
    big.grid.destroy()
    del big
    small = _grid(synth.config_c1())
    assert small.grid.n_core < 32768
    model.set_gate(_median_tau(sg, small))
    print(f"sphere64: {small.grid.n_core} core packages", flush=True)
    nf, n = _compare(sg, model, small)
    assert nf > 0
    _compare(sg, model, small, with_count=False)      # without a count pointer


def test_noalloc_arguments(sg):
    from paper_2512_11473_amd import surrogate
    wl = _grid(synth.config_c1(), n_iter=0)
    n = wl.grid.n_core * 64
    out = torch.empty((4, n), device="cuda")
    with pytest.raises(TypeError):
        sg.compute_near_surface_integrals_noalloc(wl.grid, wl.phi, out, None)
    model = sg.Mlp(surrogate.init_params(4, 2.0))
    lib = sg.load()
    st = lib.sgrid_compute_near_surface_integrals_noalloc(wl.grid.handle, wl.phi.data_ptr(), None,
                                                           out.data_ptr(), None, None)
    assert st != 0                                      # a NULL model is refused by the library
    st = lib.sgrid_compute_near_surface_integrals_noalloc(wl.grid.handle, None, model.handle,
                                                           out.data_ptr(), None, None)
    assert st != 0                                      # and so is a NULL field
    torch.cuda.synchronize()
