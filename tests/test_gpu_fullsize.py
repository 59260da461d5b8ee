"""Full-size parity (GPU): the prism512 workload exactly as bench.py runs it
(default sweep configuration, packed gradient and probe, plain integrals
direct and factorised),
compared with the oracle on every point, every particle and every core
point; the 64-shape batch in its autotuned, graph-replayed form against each
member's own sweep; and the 2048^3 displaced torus, whose tables are checked
whole and whose fields are checked on an oracle crop (a dense FP64 oracle of
the whole 2048^3 grid would need 69 GB per array)."""
import numpy as np
import pytest

import oracle
import synth
from sort_check import assert_sorted
from tables_check import assert_tables_equal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G0 = 0.865663036


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    sg.set_sweep_config(0, 1)
    return sg


def _blocked():
    loc = np.arange(64)
    i, j, k = loc % 4, (loc // 4) % 4, loc // 16
    return 8 * ((i >> 1) + 2 * (j >> 1) + 4 * (k >> 1)) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1))


def test_prism512_full_pipeline(sg):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c2()
    pos = synth.particles_for(cfg)
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    g = sg.build_packages(wl.coarse, wl.h)          # the build as the benchmark step runs it
    assert g.n_packages == 124308 and g.n_core == 56880
    sg.reinitialize(g, wl.phi, wl.scratch, cfg["n_iter"])
    packed = torch.empty((g.n_total, 64, 4), device="cuda")
    sg.compute_gradient_packed(g, wl.phi, packed)
    sg.probe_particles_packed(g, packed, wl.pos, wl.phi_p, wl.nrm_p)
    integ = torch.empty((4, g.n_core * 64), device="cuda")
    sg.compute_near_surface_integrals(g, wl.phi, integ)
    # the factorised form, as the benchmark runs it (fractions into the sweep's scratch)
    integ_f = torch.empty_like(integ)
    sg.compute_near_surface_integrals_factorised(g, wl.phi, wl.scratch, integ_f)
    torch.cuda.synchronize()
    assert torch.equal(integ_f, integ)
    del integ_f

    run = oracle.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    t = {k: v.cpu().numpy() for k, v in g.tables().items()}
    assert np.array_equal(t["cell_pkg"].view(np.uint32), run.tab.cell_pkg)
    assert np.array_equal(t["pkg_nbr"].view(np.uint32), run.tab.nbr)
    oracle.run_plain(run, cfg["n_iter"])
    h = run.h
    pts = wl.points.ravel()
    err = np.abs(wl.phi[2:].double().cpu().numpy().ravel() - run.phi[pts])
    assert err.max() <= 1e-5 * h, f"max |dphi| = {err.max() / h:.3e} h"
    unpacked = packed[:, torch.from_numpy(_blocked()).cuda(), :]
    gg = unpacked[2:, :, 1:].double().cpu().numpy().reshape(-1, 3).T
    assert np.max(np.abs(gg - run.grad[:, pts])) <= 1e-5
    ref_phi, ref_nrm, ref_g = oracle.probe(run.N, h, run.B, run.tab.cell_pkg, run.phi, run.grad,
                                           pos.astype(np.float64), with_gradient=True)
    assert np.max(np.abs(wl.phi_p.double().cpu().numpy() - ref_phi)) <= 1e-5 * h
    ok = np.linalg.norm(ref_g, axis=1) > 0.25
    assert ok.mean() > 0.95
    assert np.max(np.abs(wl.nrm_p.double().cpu().numpy()[ok] - ref_nrm[ok])) <= 1e-5
    _check_sorted_probe(sg, g, packed, wl, t, pos)
    core = t["core_list"].astype(np.int64)
    ref = oracle.integrals(run.N, h, run.B, run.phi, wl.points[core - 2].ravel())
    got = integ.double().cpu().numpy().T
    assert np.max(np.abs(got[:, 0] - ref[:, 0])) <= 1e-5
    assert np.max(np.abs(got[:, 1:] - ref[:, 1:])) <= 1e-5 * G0
    # the integral field at every activated point and its probe at all 1e7 particles (Sec. 8)
    field = torch.empty((g.n_total, 64, 4), device="cuda")
    sg.compute_integral_field(g, wl.phi, field)
    fout = torch.empty((pos.shape[0], 4), device="cuda")
    sg.probe_integral_field(g, field, wl.pos, fout)
    torch.cuda.synchronize()
    fref = oracle.integral_field(run.N, h, run.B, run.tab, run.active, run.phi)
    fgot = field[2:, torch.from_numpy(_blocked()).cuda(), :].double().cpu().numpy().reshape(-1, 4)
    fwant = fref[:, pts].T
    assert np.max(np.abs(fgot[:, 0] - fwant[:, 0])) <= 1e-5
    assert np.max(np.abs(fgot[:, 1:] - fwant[:, 1:])) <= 1e-5 * G0
    del fgot, fwant
    pref = oracle.probe_field(run.N, h, run.tab.cell_pkg, fref, pos.astype(np.float64))
    pgot = fout.double().cpu().numpy()
    assert np.max(np.abs(pgot[:, 0] - pref[:, 0])) <= 2e-5
    assert np.max(np.abs(pgot[:, 1:] - pref[:, 1:])) <= 2e-5 * G0


def test_batch64_full_size(sg):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c3()
    bw = workload.setup_batch(cfg["shapes"], cfg["noise_amp"])
    assert len(bw.parts) == 64
    bw.batch.autotune(bw.phi0, bw.scratch, reps=2)
    bw.reset()
    bw.batch.reinitialize(bw.phi, bw.scratch, cfg["n_iter"], use_graph=True)
    torch.cuda.synchronize()
    counts = np.array([p.grid.n_packages for p in bw.parts])
    pick = sorted({int(np.argmin(counts)), int(np.argmax(counts)), 7, 31, 63})
    for k in pick:
        p = bw.parts[k]
        p.reset()
        sg.reinitialize(p.grid, p.phi, p.scratch, cfg["n_iter"])
        assert torch.equal(bw.slice(k, bw.phi), p.phi), k
    # the smallest member against the oracle
    k = int(np.argmin(counts))
    spec = cfg["shapes"][k]
    run = oracle.setup(spec["shape"], spec["N"], cfg["noise_amp"], spec["noise_seed"])
    oracle.run_plain(run, cfg["n_iter"])
    got = bw.slice(k, bw.phi)[2:].double().cpu().numpy().ravel()
    assert np.max(np.abs(got - run.phi[bw.parts[k].points.ravel()])) <= 1e-5 * run.h


# 100^3 coarse cells around the top of the tube, (0.85, 0.5, 0.6)
CROP_ORIGIN = (385, 206, 257)
CROP_EXTENT = 100


def _global_rows(t, local, n, origin, M):
    """Package id and local point index, on the full grid, of crop-local fine
    indices."""
    N = 4 * M
    i = local % n + 4 * origin[0]
    j = (local // n) % n + 4 * origin[1]
    k = local // (n * n) + 4 * origin[2]
    cell = (i >> 2) + M * ((j >> 2) + M * (k >> 2))
    pkg = t["cell_pkg"].view(np.uint32)[cell].astype(np.int64)
    loc = (i & 3) + 4 * (j & 3) + 16 * (k & 3)
    return pkg, loc


def _check_sorted_probe(sg, g, packed, wl, t, pos):
    """The particle sort as the benchmark step runs it, then the probe of the
    sorted particles: every particle's bits of the generated-order probe."""
    ps = torch.empty_like(wl.pos)
    perm = torch.empty(wl.pos.shape[0], dtype=torch.int32, device="cuda")
    sg.sort_particles(g, wl.pos, ps, perm)
    php, nrp = torch.empty_like(wl.phi_p), torch.empty_like(wl.nrm_p)
    sg.probe_particles_packed(g, packed, ps, php, nrp)
    torch.cuda.synchronize()
    p = perm.long()
    assert torch.equal(php.view(torch.int32), wl.phi_p[p].view(torch.int32))
    assert torch.equal(nrp.view(torch.int32), wl.nrm_p[p].view(torch.int32))
    assert_sorted(g.n_coarse, wl.h, pos, ps.cpu().numpy(), perm.cpu().numpy())


def _interior(local, n, m):
    i, j, k = local % n, (local // n) % n, local // (n * n)
    return (i >= m) & (i < n - m) & (j >= m) & (j < n - m) & (k >= m) & (k < n - m)


@pytest.mark.timeout(900)
def test_torus2048_full_size(sg):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c5()
    N, n_iter = cfg["N"], cfg["n_iter"]
    M = N // 4
    pos = synth.particles_for(cfg)
    wl = workload.setup(cfg["shape"], N, cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    g = wl.grid
    # the worklist-ordered storage variant (which the autotuner may pick here)
    # against the default sweep, bit for bit, over a few iterations
    outs = []
    for variant in (0, 7):
        sg.set_sweep_config(variant, 1)
        wl.reset()
        sg.reinitialize(g, wl.phi, wl.scratch, 4)
        outs.append(wl.phi.clone())
    sg.set_sweep_config(0, 1)
    assert torch.equal(outs[0], outs[1])
    del outs
    wl.reset()
    sg.reinitialize(g, wl.phi, wl.scratch, n_iter)
    packed = torch.empty((g.n_total, 64, 4), device="cuda")
    sg.compute_gradient_packed(g, wl.phi, packed)
    sg.probe_particles_packed(g, packed, wl.pos, wl.phi_p, wl.nrm_p)
    integ = torch.empty((4, g.n_core * 64), device="cuda")
    sg.compute_near_surface_integrals(g, wl.phi, integ)
    integ_f = torch.empty_like(integ)
    sg.compute_near_surface_integrals_factorised(g, wl.phi, wl.scratch, integ_f)
    torch.cuda.synchronize()
    assert torch.equal(integ_f, integ)          # all 46 M core points; the crop below checks the values
    del integ_f

    # tables: the whole 512^3 background grid, bit for bit
    t = {k: v.cpu().numpy() for k, v in g.tables().items()}
    ref = oracle.build_tables(M, wl.coarse.cpu().numpy())
    assert_tables_equal(t, ref)
    del ref

    # fields: a crop, at points beyond the reach of its faces
    crop = oracle.setup_crop(cfg["shape"], N, CROP_ORIGIN, CROP_EXTENT, cfg["noise_amp"], cfg["noise_seed"])
    oracle.run_plain(crop, n_iter)
    n, h = 4 * CROP_EXTENT, crop.h
    m = n_iter + 6
    act = crop.active[_interior(crop.active, n, m)]
    assert act.size > 500_000
    pkg, loc = _global_rows(t, act, n, CROP_ORIGIN, M)
    assert np.all(pkg >= 2)                            # activated on both sides
    rows = torch.from_numpy(pkg).cuda()
    cols = torch.from_numpy(loc).cuda()
    got = wl.phi[rows, cols].double().cpu().numpy()
    assert np.max(np.abs(got - crop.phi[act])) <= 1e-5 * h
    bl = torch.from_numpy(_blocked()[loc]).cuda()
    gg = packed[rows, bl, 1:].double().cpu().numpy().T
    assert np.max(np.abs(gg - crop.grad[:, act])) <= 1e-5

    # particles whose interpolation stencil lies inside the checked region
    p64 = pos.astype(np.float64) - 4 * h * np.asarray(CROP_ORIGIN, dtype=np.float64)
    base = np.floor(p64 / h - 0.5)
    sel = np.nonzero(np.all((base >= m) & (base <= n - m - 2), axis=1))[0]
    assert sel.size > 100_000
    ref_phi, ref_nrm, ref_g = oracle.probe(n, h, crop.B, crop.tab.cell_pkg, crop.phi, crop.grad,
                                           p64[sel], with_gradient=True)
    sel_d = torch.from_numpy(sel).cuda()
    assert np.max(np.abs(wl.phi_p[sel_d].double().cpu().numpy() - ref_phi)) <= 1e-5 * h
    ok = np.linalg.norm(ref_g, axis=1) > 0.25
    assert ok.mean() > 0.95
    assert np.max(np.abs(wl.nrm_p[sel_d].double().cpu().numpy()[ok] - ref_nrm[ok])) <= 1e-5
    _check_sorted_probe(sg, g, packed, wl, t, pos)

    # integrals of the core points whose 9^3 window lies inside the checked region
    core_pts = oracle.active_points(crop.tab, (1,))
    core_pts = core_pts[_interior(core_pts, n, m + 4)]
    assert core_pts.size > 100_000
    pkg, loc = _global_rows(t, core_pts, n, CROP_ORIGIN, M)
    rank = np.searchsorted(t["core_list"].view(np.uint32).astype(np.int64), pkg)
    assert np.array_equal(t["core_list"][rank].astype(np.int64), pkg)
    col = torch.from_numpy(rank * 64 + loc).cuda()
    got = integ[:, col].double().cpu().numpy().T
    ref = oracle.integrals(n, h, crop.B, crop.phi, core_pts)
    assert np.max(np.abs(got[:, 0] - ref[:, 0])) <= 1e-5
    assert np.max(np.abs(got[:, 1:] - ref[:, 1:])) <= 1e-5 * G0


# 64^3 coarse cells across the shell's outer surface at (0.81, 0.5, 0.5)
SHELL_CROP = (175, 96, 96)
SHELL_EXTENT = 64


@pytest.mark.timeout(900)
def test_shell1024_full_size(sg):
    """The paper's timing geometry at its resolution: tables bit for bit, the
    sequential update exactly, the Laplacian on an oracle crop."""
    from paper_2512_11473_amd import workload
    cfg = synth.config_shell()
    N = cfg["N"]
    M = N // 4
    wl = workload.setup(cfg["shape"], N, cfg["noise_amp"], cfg["noise_seed"])
    g = wl.grid
    assert g.n_packages == 579128
    out = torch.empty_like(wl.phi)
    sg.compute_laplacian(g, wl.phi, out)
    before = wl.phi.clone()
    sg.sequential_update(g, wl.phi, cfg["delta"])
    torch.cuda.synchronize()
    assert torch.equal(wl.phi[2:], before[2:] + torch.tensor(cfg["delta"], dtype=torch.float32, device="cuda"))
    t = {k: v.cpu().numpy() for k, v in g.tables().items()}
    assert_tables_equal(t, oracle.build_tables(M, wl.coarse.cpu().numpy()))
    crop = oracle.setup_crop(cfg["shape"], N, SHELL_CROP, SHELL_EXTENT, cfg["noise_amp"], cfg["noise_seed"])
    n, h = 4 * SHELL_EXTENT, crop.h
    dense = oracle.dense_state(crop.tab, crop.active, crop.phi0, crop.B)
    ref = oracle.laplacian(n, h, crop.B, crop.active, dense)
    act = crop.active[_interior(crop.active, n, 6)]
    assert act.size > 200_000
    pkg, loc = _global_rows(t, act, n, SHELL_CROP, M)
    assert np.all(pkg >= 2)
    got = out[torch.from_numpy(pkg).cuda(), torch.from_numpy(loc).cuda()].double().cpu().numpy()
    assert np.max(np.abs(got - ref[act])) <= 3e-5 / h
