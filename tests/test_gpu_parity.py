"""Parity of the HIP path against the FP64 oracle (GPU).

Tables must match bit for bit; fields within the tolerances the method
states: |dphi| <= 1e-5 h (FP32 against FP64), 1e-12 h for the FP64 kernels;
gradients and normals (unitless) 1e-5; integrals 1e-5 (K_W) and 1e-5 G0 (h K_grad).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tables_check import assert_tables_equal as _assert_tables_equal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G0 = 0.865663036   # h * K_grad of an axis-aligned half-space through the query point


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    sg.set_sweep_config(0, 1)
    return sg


def _gpu_tables(sg, d, h):
    g = sg.build_packages(torch.from_numpy(d).cuda(), h)
    t = {k: v.cpu().numpy() for k, v in g.tables().items()}
    return g, t


# --------------------------------------------------------------------------
# Tables (bit-exact)
# --------------------------------------------------------------------------

def test_tables_all_core_patterns_m2(sg):
    M = 2
    rng = np.random.default_rng(0)
    for pattern in range(256):
        core = np.array([(pattern >> c) & 1 for c in range(8)], dtype=bool)
        d = np.where(core, rng.uniform(-0.49, 0.49, 8), rng.choice([-1, 1], 8) * rng.uniform(0.5, 2, 8))
        d = d.astype(np.float32)
        g, t = _gpu_tables(sg, d, 1.0 / (4 * M))
        _assert_tables_equal(t, oracle.build_tables(M, d))
        g.destroy()


@pytest.mark.parametrize("M", [1, 3, 5, 8, 13, 32])
def test_tables_random_with_ties(sg, M):
    rng = np.random.default_rng(M)
    lc = 1.0 / M
    for _ in range(5):
        d = (rng.uniform(-3, 3, M ** 3) * lc).astype(np.float32)
        d[rng.uniform(size=M ** 3) < 0.1] = np.float32(lc)
        d[rng.uniform(size=M ** 3) < 0.05] = np.float32(-lc)
        d[rng.uniform(size=M ** 3) < 0.05] = np.float32(-0.0)
        g, t = _gpu_tables(sg, d, 1.0 / (4 * M))
        _assert_tables_equal(t, oracle.build_tables(M, d))


@pytest.mark.parametrize("cfg", [synth.config_c1(), synth.config_c2()], ids=["sphere64", "prism512"])
def test_tables_named_workloads(sg, cfg):
    M = cfg["N"] // 4
    d = synth.coarse_sdf(cfg["shape"], M)
    g, t = _gpu_tables(sg, d, 1.0 / cfg["N"])
    _assert_tables_equal(t, oracle.build_tables(M, d))


def test_tables_random_unions(sg):
    for s in synth.batch_shapes(6, 11, resolutions=(64, 128)):
        M = s["N"] // 4
        d = synth.coarse_sdf(s["shape"], M)
        g, t = _gpu_tables(sg, d, 1.0 / s["N"])
        _assert_tables_equal(t, oracle.build_tables(M, d))


def test_empty_band(sg):
    M = 6
    d = np.full(M ** 3, 10.0, dtype=np.float32)
    g, t = _gpu_tables(sg, d, 1.0 / (4 * M))
    assert g.n_packages == 0 and g.n_core == 0
    assert np.all(t["cell_pkg"] == 1)
    phi = g.empty_field()
    sg.fill_far_field(g, phi)
    scratch = torch.empty_like(phi)
    sg.reinitialize(g, phi, scratch, 3)
    grad = g.empty_field(components=3)
    sg.compute_gradient(g, phi, grad)
    pos = torch.rand(100, 3, device="cuda")
    po, no = torch.empty(100, device="cuda"), torch.empty(100, 3, device="cuda")
    sg.probe_particles(g, phi, grad, pos, po, no)
    out = torch.empty(0, device="cuda")
    sg.compute_near_surface_integrals(g, phi, out)
    torch.cuda.synchronize()
    assert torch.allclose(po, torch.full_like(po, 16 * g.h), rtol=1e-6, atol=0) and torch.all(no == 0)
    assert torch.all(grad == 0)


# --------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------

def _ulp32(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


def _run_both(sg, cfg, dtype, n_iter, n_particles=None):
    from paper_2512_11473_amd import workload
    N = cfg["N"]
    pos = synth.particles_for(cfg, n_particles) if n_particles else None
    wl = workload.setup(cfg["shape"], N, cfg["noise_amp"], cfg["noise_seed"], dtype=dtype, particles=pos)
    run = oracle.setup(cfg["shape"], N, cfg["noise_amp"], cfg["noise_seed"],
                       phi0_dtype=np.float32 if dtype == torch.float32 else np.float64)
    return wl, run, pos


@pytest.mark.parametrize("dtype,tol_h", [(torch.float32, 1e-5), (torch.float64, 1e-12)], ids=["f32", "f64"])
def test_sphere64_pipeline(sg, dtype, tol_h):
    cfg = synth.config_c1()
    wl, run, pos = _run_both(sg, cfg, dtype, cfg["n_iter"], cfg["n_particles"])
    h = wl.h
    pts = wl.points.ravel()
    # one iteration: a few units in the last place
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, 1)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    one = oracle.reinit(run.N, h, run.B, run.active, dense, 1)
    got = wl.phi[2:].double().cpu().numpy().ravel()
    if dtype == torch.float32:
        assert np.all(np.abs(got - one[pts]) <= 4 * _ulp32(one[pts]) + 2e-7 * h)
    else:
        assert np.max(np.abs(got - one[pts])) <= tol_h * h
    # far-field rows are never written
    assert torch.all(wl.phi[0] == -16 * h) and torch.all(wl.phi[1] == 16 * h)
    # the full iteration count
    wl.reset()
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, cfg["n_iter"])
    oracle.run_plain(run, cfg["n_iter"])
    got = wl.phi[2:].double().cpu().numpy().ravel()
    err = np.abs(got - run.phi[pts])
    assert err.max() <= tol_h * h, f"max |dphi| = {err.max() / h:.3e} h"
    # gradient
    sg.compute_gradient(wl.grid, wl.phi, wl.grad)
    gg = wl.grad[:, 2:].double().cpu().numpy().reshape(3, -1)
    gtol = 1e-5 if dtype == torch.float32 else 1e-11
    assert np.max(np.abs(gg - run.grad[:, pts])) <= gtol
    assert torch.all(wl.grad[:, :2] == 0)
    # probe
    sg.probe_particles(wl.grid, wl.phi, wl.grad, wl.pos, wl.phi_p, wl.nrm_p)
    ref_phi, ref_nrm, ref_g = oracle.probe(run.N, h, run.B, run.tab.cell_pkg, run.phi, run.grad,
                                           pos.astype(np.float64), with_gradient=True)
    pp = wl.phi_p.double().cpu().numpy()
    nn = wl.nrm_p.double().cpu().numpy()
    assert np.max(np.abs(pp - ref_phi)) <= tol_h * h
    ok = np.linalg.norm(ref_g, axis=1) > 0.25   # normals are ill-conditioned where g vanishes
    assert ok.mean() > 0.95
    assert np.max(np.abs(nn[ok] - ref_nrm[ok])) <= (1e-5 if dtype == torch.float32 else 1e-11)
    far = np.linalg.norm(ref_g, axis=1) == 0
    assert np.all(nn[far] == 0)
    # packed (phi, g) layout gives identical probe results
    packed = torch.empty((wl.grid.n_total, 64, 4), dtype=dtype, device="cuda")
    sg.compute_gradient_packed(wl.grid, wl.phi, packed)
    loc = np.arange(64)
    i, j, k = loc % 4, (loc // 4) % 4, loc // 16
    blk = torch.from_numpy(8 * ((i >> 1) + 2 * (j >> 1) + 4 * (k >> 1)) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1))).cuda()
    unpacked = packed[:, blk, :]             # back to the i + 4j + 16k order
    assert torch.equal(unpacked[..., 0], wl.phi)
    assert torch.equal(unpacked[..., 1:].permute(2, 0, 1), wl.grad)
    pp2, nn2 = torch.empty_like(wl.phi_p), torch.empty_like(wl.nrm_p)
    sg.probe_particles_packed(wl.grid, packed, wl.pos, pp2, nn2)
    assert torch.equal(pp2, wl.phi_p) and torch.equal(nn2, wl.nrm_p)


def test_sphere64_gradient_on_initial_field(sg):
    cfg = synth.config_c1()
    wl, run, _ = _run_both(sg, cfg, torch.float32, 0)
    sg.compute_gradient(wl.grid, wl.phi, wl.grad)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    ref = oracle.gradient(run.N, run.h, run.B, run.active, dense)
    gg = wl.grad[:, 2:].double().cpu().numpy().reshape(3, -1)
    assert np.max(np.abs(gg - ref[:, wl.points.ravel()])) <= 1e-6


def _core_points(wl):
    """Fine indices of the core points in output order [n_core * 64]."""
    t = wl.grid.tables()
    core = t["core_list"].cpu().numpy().astype(np.int64)
    return wl.points[core - 2].ravel()


@pytest.mark.parametrize("n_iter", [0, 20])
def test_sphere64_integrals(sg, n_iter):
    cfg = synth.config_c1()
    wl, run, _ = _run_both(sg, cfg, torch.float32, n_iter)
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
    oracle.run_plain(run, n_iter)
    out = torch.empty((4, wl.grid.n_core * 64), device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    sg.compute_near_surface_integrals(wl.grid, wl.phi, out, n_fallback=nf)
    ref = oracle.integrals(run.N, run.h, run.B, run.phi, _core_points(wl))
    got = out.double().cpu().numpy().T
    assert int(nf.item()) == 0
    assert np.max(np.abs(got[:, 0] - ref[:, 0])) <= 1e-5
    assert np.max(np.abs(got[:, 1:] - ref[:, 1:])) <= 1e-5 * G0
    # the band holds both saturated and cut cells
    assert (ref[:, 0] > 0.01).mean() > 0.2 and (ref[:, 0] < 0.97).mean() > 0.2


@pytest.mark.parametrize("n_iter", [0, 20])
@pytest.mark.parametrize("variant", [0, 3], ids=["id-order", "morton-order"])
def test_sphere64_integrals_factorised(sg, n_iter, variant):
    """The two-pass integrals (cut fractions at every point, then the taps)
    against the oracle, and bit for bit against the direct kernel; the first
    pass runs in package-id or Morton order as the sweep setting says."""
    cfg = synth.config_c1()
    wl, run, _ = _run_both(sg, cfg, torch.float32, n_iter)
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
    oracle.run_plain(run, n_iter)
    n = wl.grid.n_core * 64
    direct = torch.empty((4, n), device="cuda")
    fact = torch.full((4, n), float("nan"), device="cuda")
    vfrac = torch.full_like(wl.phi, float("nan"))
    sg.set_sweep_config(variant, 1)
    try:
        sg.compute_near_surface_integrals(wl.grid, wl.phi, direct)
        sg.compute_near_surface_integrals_factorised(wl.grid, wl.phi, vfrac, fact)
        torch.cuda.synchronize()
    finally:
        sg.set_sweep_config(0, 1)
    assert torch.equal(fact, direct)
    ref = oracle.integrals(run.N, run.h, run.B, run.phi, _core_points(wl))
    got = fact.double().cpu().numpy().T
    assert np.max(np.abs(got[:, 0] - ref[:, 0])) <= 1e-5
    assert np.max(np.abs(got[:, 1:] - ref[:, 1:])) <= 1e-5 * G0
    # the fractions of the first pass: far-field rows 0 and 1, band points in [0, 1]
    v = vfrac.cpu()
    assert torch.all(v[0] == 0) and torch.all(v[1] == 1)
    assert torch.all((v[2:] >= 0) & (v[2:] <= 1))


def test_integrals_factorised_domain_faces(sg):
    """Core packages whose window reaches out of the domain (far-field
    neighbours) take the in-kernel fraction path; the result is still the
    direct kernel's bits and the oracle's values."""
    from paper_2512_11473_amd import workload
    s = synth.union([synth.sphere((0.14, 0.5, 0.5), 0.12), synth.box((0.6, 0.8, 0.5), (0.25, 0.16, 0.25))])
    N = 64
    wl = workload.setup(s, N, 0.1, 21)
    run = oracle.setup(s, N, 0.1, 21)
    t = {k: v.cpu().numpy() for k, v in wl.grid.tables().items()}
    nbr = t["pkg_nbr"].view(np.uint32)
    core = t["core_list"].astype(np.int64)
    edge = np.any(nbr[core] < 2, axis=1)
    assert edge.any() and not edge.all()                    # some core windows leave the domain, some do not
    # a second-pass wavefront takes four consecutive core packages: some take
    # both kinds, and the last (a partial one) takes domain-face packages
    groups = [edge[i:i + 4] for i in range(0, edge.size, 4)]
    assert any(gr.any() and not gr.all() for gr in groups)
    assert edge.size % 4 != 0 and groups[-1].any()
    n = wl.grid.n_core * 64
    direct = torch.empty((4, n), device="cuda")
    fact = torch.empty((4, n), device="cuda")
    vfrac = torch.empty_like(wl.phi)
    for n_iter in (0, 3):
        if n_iter:
            sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
        oracle.run_plain(run, n_iter)
        sg.compute_near_surface_integrals(wl.grid, wl.phi, direct)
        sg.compute_near_surface_integrals_factorised(wl.grid, wl.phi, vfrac, fact)
        torch.cuda.synchronize()
        assert torch.equal(fact, direct), n_iter
        ref = oracle.integrals(run.N, run.h, run.B, run.phi, wl.points[core - 2].ravel())
        got = fact.double().cpu().numpy().T
        assert np.max(np.abs(got[:, 0] - ref[:, 0])) <= 1e-5, n_iter
        assert np.max(np.abs(got[:, 1:] - ref[:, 1:])) <= 1e-5 * G0, n_iter


def test_integrals_factorised_ragged_and_empty(sg):
    """Core counts that leave the last workgroup partly empty (the second pass
    takes four core packages per wavefront and sixteen per workgroup, so
    counts of 6 and 14 mod 16 leave a wavefront with two), and a grid with no
    core package at all (a call that launches nothing)."""
    from paper_2512_11473_amd import workload
    seen = set()
    for r, seed in ((0.11, 3), (0.17, 4), (0.23, 5), (0.29, 6)):
        wl = workload.setup(synth.sphere((0.5, 0.47, 0.52), r), 64, 0.1, seed)
        n = wl.grid.n_core * 64
        seen.add(wl.grid.n_core % 16)
        direct = torch.empty((4, n), device="cuda")
        fact = torch.empty((4, n), device="cuda")
        sg.compute_near_surface_integrals(wl.grid, wl.phi, direct)
        sg.compute_near_surface_integrals_factorised(wl.grid, wl.phi, torch.empty_like(wl.phi), fact)
        torch.cuda.synchronize()
        assert torch.equal(fact, direct)
    assert any(x % 4 for x in seen)
    d = torch.full((8 ** 3,), 1.0, device="cuda")           # every coarse cell far outside: P = 0
    g = sg.build_packages(d, 1.0 / 32)
    assert g.n_core == 0
    phi = torch.zeros((g.n_total, 64), device="cuda")
    sg.compute_near_surface_integrals_factorised(g, phi, torch.zeros_like(phi), torch.empty((4, 0), device="cuda"))
    torch.cuda.synchronize()
    g.destroy()


def test_integrals_every_point_cut(sg):
    """phi = 0 at every band point: every cut fraction is 1/2 (zero gradient,
    a = 0), so every point of every window goes through the listed-point path
    of both forms (full lists: 256 points per first-pass wavefront, 343 per
    direct window).  By symmetry K_grad is exactly 0 and K_W is half the full
    kernel sum."""
    from paper_2512_11473_amd import workload
    wl = workload.setup(synth.sphere((0.5, 0.47, 0.52), 0.23), 64, 0.1, 5)
    phi = wl.phi.clone()
    phi[2:] = 0.0                                           # far-field rows keep -B / +B
    n = wl.grid.n_core * 64
    direct = torch.empty((4, n), device="cuda")
    fact = torch.empty((4, n), device="cuda")
    sg.compute_near_surface_integrals(wl.grid, phi, direct)
    sg.compute_near_surface_integrals_factorised(wl.grid, phi, torch.empty_like(phi), fact)
    torch.cuda.synchronize()
    assert torch.equal(fact, direct)
    got = direct.double().cpu().numpy()
    assert np.all(got[1:] == 0.0)
    assert np.max(np.abs(got[0] - 0.5 * oracle.c_full())) <= 1e-6


def test_sweep_variants_identical(sg):
    cfg = synth.config_c1()
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    results = []
    for variant, groups in [(0, 1), (0, 2), (0, 3), (0, 4), (0, 8), (1, 1), (1, 2), (1, 3), (2, 1), (2, 2), (2, 4), (2, 8),
                           (3, 1), (3, 2), (3, 4), (4, 1), (5, 1), (5, 2), (5, 4), (6, 1), (6, 3), (6, 8), (7, 1)]:
        sg.set_sweep_config(variant, groups)
        wl.reset()
        sg.reinitialize(wl.grid, wl.phi, wl.scratch, 7)
        results.append(wl.phi.clone())
    sg.set_sweep_config(0, 1)
    for r in results[1:]:
        assert torch.equal(r, results[0])


def test_worklist_storage_sweep_iteration_counts(sg):
    """Variant 7 holds the field in worklist order between its first and last
    sweep: one sweep (id order to id order), two (gather then scatter), and
    odd and even longer counts (the last result copied back when it lands in
    the scratch buffer) all give the bits of the default sweep, and leave the
    far-field rows untouched."""
    from paper_2512_11473_amd import workload
    prism128 = {"shape": synth.prism(), "N": 128, "noise_amp": 0.05, "noise_seed": 3}
    for cfg in (synth.config_c1(), prism128):
        wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
        for n_iter in (1, 2, 3, 4, 9):
            out = []
            for variant in (0, 7):
                sg.set_sweep_config(variant, 1)
                wl.reset()
                sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
                out.append(wl.phi.clone())
            sg.set_sweep_config(0, 1)
            assert torch.equal(out[1], out[0]), n_iter
            assert torch.all(out[1][0] == -16 * wl.h) and torch.all(out[1][1] == 16 * wl.h)


def test_persistent_sweep_rounds(sg):
    """The persistent worklist sweep over a grid that takes each wavefront
    through several grid-stride rounds, with a ragged last set, gives the bits
    of the one-shot sweeps."""
    from paper_2512_11473_amd import workload
    wl = workload.setup(synth.sphere((0.48, 0.51, 0.49), 0.33), 256, 0.1, 5)
    P = wl.grid.n_packages
    assert (P + 3) // 4 > 3 * 256 * 4 and P % 4 != 0      # more than three rounds at one workgroup per CU
    results = []
    for variant, groups in [(0, 1), (3, 1), (2, 1), (2, 2), (2, 3), (2, 8), (6, 1), (6, 4)]:
        sg.set_sweep_config(variant, groups)
        wl.reset()
        sg.reinitialize(wl.grid, wl.phi, wl.scratch, 5)
        results.append(wl.phi.clone())
    sg.set_sweep_config(0, 1)
    for r in results[1:]:
        assert torch.equal(r, results[0])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_sweep_domain_edge(sg, dtype):
    """A band cut by two domain faces (out-of-domain neighbours are the
    positive far field) with far field on both sides, every sweep variant,
    even and odd iteration counts.  The shapes' interiors stay clear of the
    faces: where an interior touches a face, its points see the +B far field
    across it, the update there jumps by several h per iteration, and FP32
    rounding is amplified beyond 1e-5 h within a few iterations (a property of
    the iteration, not of the kernels: tests/test_fp32_domain_face.py shows it
    with a correctly rounded FP32 evaluation of the update)."""
    from paper_2512_11473_amd import workload
    s = synth.union([synth.sphere((0.14, 0.5, 0.5), 0.12), synth.box((0.6, 0.8, 0.5), (0.25, 0.16, 0.25))])
    N = 64
    wl = workload.setup(s, N, 0.1, 21, dtype=dtype)
    run = oracle.setup(s, N, 0.1, 21, phi0_dtype=np.float32 if dtype == torch.float32 else np.float64)
    tab = {k: v.cpu().numpy() for k, v in wl.grid.tables().items()}
    nbr = tab["pkg_nbr"].view(np.uint32)
    cells = tab["pkg_cell"].view(np.uint32)[2:].astype(np.int64)
    M = N // 4
    x, y = cells % M, (cells // M) % M
    assert np.any(x == 0) and np.any(y == M - 1)           # the band reaches both faces
    assert np.any(nbr[2:] == 0) and np.any(nbr[2:] == 1)    # far field on both sides
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    configs = [(0, 1), (0, 4), (1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (6, 2)]
    for n_iter in (1, 2, 5, 12):
        outs = []
        for variant, groups in configs:
            sg.set_sweep_config(variant, groups)
            wl.reset()
            sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
            outs.append(wl.phi.clone())
        sg.set_sweep_config(0, 1)
        for o in outs[1:]:
            assert torch.equal(outs[0], o), n_iter
        phi = oracle.reinit(run.N, run.h, run.B, run.active,
                            oracle.dense_state(run.tab, run.active, run.phi0, run.B), n_iter)
        got = outs[0][2:].double().cpu().numpy().ravel()
        assert np.max(np.abs(got - phi[wl.points.ravel()])) <= tol * run.h, n_iter


def test_sweep_autotune(sg):
    """The sweep autotuner times its candidates, leaves phi untouched, picks
    one of them, and the tuned sweep gives the bits of the default one."""
    cfg = synth.config_c1()
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, 3)
    ref = wl.phi.clone()
    before = wl.phi.clone()
    v, g, table = sg.autotune_sweep(wl.grid, wl.phi, wl.scratch, reps=2)
    assert torch.equal(wl.phi, before)
    assert (v, g) in sg.SWEEP_TUNE_CANDIDATES
    assert np.all(table > 0)
    wl.reset()
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, 3)
    sg.set_sweep_config(0, 1)
    assert torch.equal(wl.phi, ref)


LAP_TOL = 3e-5   # |dL| * h: FP32 sums of seven values of magnitude <= 16 h, times the exact 1 / h^2


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("which", ["sphere64", "shell128"])
def test_timing_operations(sg, dtype, which):
    """The two operations of the paper's timing test (Sec. 9, Tab. 1): the
    sequential update is the same floating-point addition as on the host, the
    seven-point Laplacian matches the oracle."""
    from paper_2512_11473_amd import workload
    if which == "sphere64":
        cfg = synth.config_c1()
        shape, N, amp, seed = cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"]
    else:
        shape, N, amp, seed = synth.shell((0.5, 0.5, 0.5), 0.3, 0.34), 128, 0.05, 8
    npd = np.float32 if dtype == torch.float32 else np.float64
    wl = workload.setup(shape, N, amp, seed, dtype=dtype)
    run = oracle.setup(shape, N, amp, seed, phi0_dtype=npd)
    out = torch.empty_like(wl.phi)
    sg.compute_laplacian(wl.grid, wl.phi, out)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    ref = oracle.laplacian(run.N, run.h, run.B, run.active, dense)
    got = out[2:].double().cpu().numpy().ravel()
    tol = LAP_TOL / run.h if dtype == torch.float32 else 1e-9 / run.h
    assert np.max(np.abs(got - ref[wl.points.ravel()])) <= tol
    assert torch.all(out[:2] == 0)
    # the far field is visible to part of the band
    assert np.abs(ref[wl.points.ravel()]).max() > 10 / run.h
    before = wl.phi.clone()
    sg.sequential_update(wl.grid, wl.phi, 1e-6)
    expect = before[2:] + torch.tensor(1e-6, dtype=dtype, device="cuda")
    assert torch.equal(wl.phi[2:], expect)
    assert torch.equal(wl.phi[:2], before[:2])


def test_stencils_in_sweep_order(sg):
    """With a Morton-order sweep configured, the gradient and the Laplacian
    visit the packages in that order too; the results are the same bits."""
    cfg = synth.config_c1()
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, 4)
    outs = []
    for variant in (0, 2, 3, 4):
        sg.set_sweep_config(variant, 1)
        grad = torch.empty((3,) + tuple(wl.phi.shape), device="cuda")
        packed = torch.empty((wl.grid.n_total, 64, 4), device="cuda")
        lap = torch.empty_like(wl.phi)
        sg.compute_gradient(wl.grid, wl.phi, grad)
        sg.compute_gradient_packed(wl.grid, wl.phi, packed)
        sg.compute_laplacian(wl.grid, wl.phi, lap)
        outs.append((grad, packed, lap))
    sg.set_sweep_config(0, 1)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_determinism(sg):
    cfg = synth.config_c1()
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"],
                        particles=synth.particles_for(cfg, 5000))
    outs = []
    for _ in range(2):
        wl.reset()
        sg.reinitialize(wl.grid, wl.phi, wl.scratch, 5)
        sg.compute_gradient(wl.grid, wl.phi, wl.grad)
        sg.probe_particles(wl.grid, wl.phi, wl.grad, wl.pos, wl.phi_p, wl.nrm_p)
        out = torch.empty((4, wl.grid.n_core * 64), device="cuda")
        sg.compute_near_surface_integrals(wl.grid, wl.phi, out)
        outs.append([wl.phi.clone(), wl.grad.clone(), wl.phi_p.clone(), wl.nrm_p.clone(), out])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_probe_edge_positions(sg):
    # particles outside the domain, on cell faces, at NaN: clamped, never out of bounds
    cfg = synth.config_c1()
    pos = np.array([[-0.3, 0.5, 0.5], [1.7, 0.5, 0.5], [0.5, 0.5, 0.25], [0.0, 0.0, 0.0],
                    [1.0, 1.0, 1.0], [0.2, 0.5, 0.5], [0.8, 0.8, 0.2]], dtype=np.float32)
    wl, run, _ = _run_both(sg, cfg, torch.float32, 0)
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    sg.compute_gradient(wl.grid, wl.phi, wl.grad)
    sg.probe_particles(wl.grid, wl.phi, wl.grad, wl.pos, wl.phi_p, wl.nrm_p)
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    g = oracle.gradient(run.N, run.h, run.B, run.active, dense)
    ref, nrm = oracle.probe(run.N, run.h, run.B, run.tab.cell_pkg, dense, g, pos.astype(np.float64))
    assert np.max(np.abs(wl.phi_p.double().cpu().numpy() - ref)) <= 1e-5 * run.h
    nanpos = torch.tensor([[float("nan"), 0.5, 0.5]], device="cuda")
    po, no = torch.empty(1, device="cuda"), torch.empty(1, 3, device="cuda")
    sg.probe_particles(wl.grid, wl.phi, wl.grad, nanpos, po, no)
    torch.cuda.synchronize()
