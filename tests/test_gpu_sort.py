"""The particle sort by home cell (GPU) and the probe on sorted particles.

The sort is a stable radix sort on the Morton code of each particle's home
coarse cell, so its permutation is unique: it must equal the stable argsort
of the keys recomputed on the host in the kernel's FP32 arithmetic, and the
sorted positions must be the input's bit for bit.  The probe of the sorted
particles must give every particle the bits the probe in generated order
gives it, and the oracle's values.
"""
import numpy as np
import pytest

import oracle
import synth
from sort_check import assert_sorted

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    return sg


def _tables(grid):
    return {k: v.cpu().numpy() for k, v in grid.tables().items()}


def _sort(sg, grid, pos, ws=None):
    pt = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float32)).cuda()
    ps = torch.empty_like(pt)
    perm = torch.empty(pt.shape[0], dtype=torch.int32, device="cuda")
    sg.sort_particles(grid, pt, ps, perm, workspace=ws)
    torch.cuda.synchronize()
    return pt, ps, perm


EDGE = np.array([[-0.3, 0.5, 0.5], [1.7, 0.5, 0.5], [0.5, 0.5, 0.25], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0],
                 [0.2, 0.5, 0.5], [0.8, 0.8, 0.2], [0.5, 0.5, 0.8], [float("nan"), 0.5, 0.5],
                 [0.5, float("inf"), 0.5]], dtype=np.float32)


def test_sort_sphere64_and_probe(sg):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c1()
    pos = np.concatenate([synth.particles_for(cfg), EDGE])
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, cfg["n_iter"])
    packed = torch.empty((wl.grid.n_total, 64, 4), device="cuda")
    sg.compute_gradient_packed(wl.grid, wl.phi, packed)
    M = wl.grid.n_coarse
    pt, ps, perm = _sort(sg, wl.grid, pos)
    keys = assert_sorted(M, wl.h, pos, ps.cpu().numpy(), perm.cpu().numpy())
    assert len(np.unique(keys)) > 1000                     # particles spread over the band's packages
    # the probe of the sorted particles: each particle's bits of the generated-order probe
    sg.probe_particles_packed(wl.grid, packed, wl.pos, wl.phi_p, wl.nrm_p)
    php, nrp = torch.empty_like(wl.phi_p), torch.empty_like(wl.nrm_p)
    sg.probe_particles_packed(wl.grid, packed, ps, php, nrp)
    torch.cuda.synchronize()
    p = perm.long()
    assert torch.equal(php.view(torch.int32), wl.phi_p[p].view(torch.int32))
    assert torch.equal(nrp.view(torch.int32), wl.nrm_p[p].view(torch.int32))
    # and the oracle's values at the sorted positions (finite ones)
    run = oracle.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    oracle.run_plain(run, cfg["n_iter"])
    psn = ps.cpu().numpy().astype(np.float64)
    fin = np.all(np.isfinite(psn), axis=1)
    ref, _ = oracle.probe(run.N, run.h, run.B, run.tab.cell_pkg, run.phi, run.grad, psn[fin])
    assert np.max(np.abs(php.cpu().numpy()[fin] - ref)) <= 1e-5 * run.h


def test_sort_edge_cases(sg):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c1()
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    M = wl.grid.n_coarse
    ws = torch.empty(sg.sort_workspace_bytes(wl.grid, 1 << 20), dtype=torch.uint8, device="cuda")
    # nothing to sort
    empty = torch.empty((0, 3), device="cuda")
    sg.sort_particles(wl.grid, empty, torch.empty_like(empty), torch.empty(0, dtype=torch.int32, device="cuda"),
                      workspace=ws)
    rng = np.random.default_rng(7)
    cases = {
        "one": np.array([[0.5, 0.5, 0.2]], dtype=np.float32),
        # every particle in one package: one bin takes all the atomics
        "one package": (0.5 + 0.25 * rng.random((4099, 3)) / 64 + np.array([0.0, 0.0, -0.3])).astype(
            np.float32),
        # every particle in the positive far field
        "far field": (0.02 + 0.05 * rng.random((777, 3))).astype(np.float32),
        # ragged counts over the whole box, the same workspace reused
        "box 257": rng.random((257, 3)).astype(np.float32),
        "box 65537": rng.random((65537, 3)).astype(np.float32),
        # many equal keys in a ragged count: the stable order decides
        "eight cells 9999": (np.floor(rng.random((9999, 3)) * 2) * 0.5 + 0.01).astype(np.float32),
    }
    for name, pos in cases.items():
        pt, ps, perm = _sort(sg, wl.grid, pos, ws)
        keys = assert_sorted(M, wl.h, pos, ps.cpu().numpy(), perm.cpu().numpy())
        if name == "one package":
            assert len(np.unique(keys)) == 1
        if name == "eight cells 9999":
            assert len(np.unique(keys)) == 8
    # argument checks
    pos = cases["box 257"]
    pt = torch.from_numpy(pos).cuda()
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    out, perm = torch.empty_like(pt), torch.empty(257, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        sg.sort_particles(wl.grid, pt, out, perm, workspace=small)
    st = sg.load().sgrid_sort_particles(wl.grid.handle, pt.data_ptr(), 257, out.data_ptr(), perm.data_ptr(),
                                        small.data_ptr(), 8, None)
    assert st == 1                                          # the library's own size check
    with pytest.raises(sg.SgridError):
        sg.sort_particles(wl.grid, pt, pt, torch.empty(257, dtype=torch.int32, device="cuda"), workspace=ws)
    with pytest.raises(TypeError):
        sg.sort_particles(wl.grid, pt, torch.empty_like(pt), torch.empty(257, dtype=torch.int64, device="cuda"))


def test_sort_keys_follow_worklist(sg):
    """Particles placed one per activated package at the package centre come
    out in the sweep worklist's order of their packages (both are the Morton
    order of the coarse cells)."""
    from paper_2512_11473_amd import workload
    cfg = synth.config_c1()
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    t = _tables(wl.grid)
    M = wl.grid.n_coarse
    cells = t["pkg_cell"].view(np.uint32)[2:].astype(np.int64)
    centre = np.stack([cells % M, (cells // M) % M, cells // (M * M)], axis=1) * (4 * wl.h) + 2 * wl.h
    pos = centre[::-1].astype(np.float32)                  # reversed id order
    pt, ps, perm = _sort(sg, wl.grid, pos)
    keys = assert_sorted(M, wl.h, pos, ps.cpu().numpy(), perm.cpu().numpy())
    assert np.all(np.diff(keys) > 0)                       # one particle per cell
    order = t["sweep_order"].view(np.uint32).astype(np.int64)
    assert np.array_equal(cells.size - 1 - perm.cpu().numpy().astype(np.int64), order - 2)


def test_sort_single_pass(sg):
    """At 8 coarse cells per axis the Morton key has 9 bits: one pass, which
    both computes the keys and gathers the sorted positions.  (Two passes run
    at 16 cells per axis above, three at 128 and 512 in the full-size tests.)"""
    from paper_2512_11473_amd import workload
    wl = workload.setup(synth.sphere(), 32, 0.1, 1)
    M = wl.grid.n_coarse
    assert M == 8
    rng = np.random.default_rng(11)
    for n in (1, 4096, 4097, 30001):
        pos = rng.random((n, 3)).astype(np.float32)
        pt, ps, perm = _sort(sg, wl.grid, pos)
        keys = assert_sorted(M, wl.h, pos, ps.cpu().numpy(), perm.cpu().numpy())
        if n == 30001:
            assert len(np.unique(keys)) == M ** 3             # every cell of the box holds particles
