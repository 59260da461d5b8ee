"""The integral field and its grid-to-particle probe (Sec. 8) against the
oracle: the field at every activated point, the one-sided far-field rows, and
the interpolated field at particles, including particles whose home cell is
far field and positions on the domain faces."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

G0 = 0.865663036   # h * K_grad of an axis-aligned half-space through the query point


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2512_11473_amd as sg
    sg.load()
    sg.set_sweep_config(0, 1)
    return sg


def _blocked():
    loc = np.arange(64)
    i, j, k = loc % 4, (loc // 4) % 4, loc // 16
    return 8 * ((i >> 1) + 2 * (j >> 1) + 4 * (k >> 1)) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1))


def _setup(sg, cfg, n_iter, pos):
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    run = oracle.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], phi0_dtype=np.float32)
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
    oracle.run_plain(run, n_iter)
    return wl, run


@pytest.mark.parametrize("which", ["sphere64", "shell128"])
def test_integral_field_and_probe(sg, which):
    if which == "sphere64":
        cfg = synth.config_c1()
        n_iter = cfg["n_iter"]
    else:
        cfg = {"shape": synth.shell((0.5, 0.5, 0.5), 0.3, 0.34), "N": 128, "noise_amp": 0.05, "noise_seed": 8}
        n_iter = 10
    N = cfg["N"]
    rng = np.random.default_rng(17)
    # particles around the surface, uniform in the domain, on data points and
    # on the domain faces and corners
    near = synth.particles_for(synth.config_c1(), 4000) if which == "sphere64" else \
        (rng.random((4000, 3)) * 0.8 + 0.1).astype(np.float32)
    unif = rng.random((2000, 3)).astype(np.float32)
    onpt = ((rng.integers(0, N, (500, 3)) + 0.5) / N).astype(np.float32)
    faces = np.array([[0, 0, 0], [1, 1, 1], [0, 0.5, 0.5], [1, 0.5, 0.5], [0.5, 0, 1], [-0.2, 0.5, 0.5],
                      [1.3, 0.2, 0.9]], dtype=np.float32)
    pos = np.concatenate([near, unif, onpt, faces])
    wl, run = _setup(sg, cfg, n_iter, pos)
    field = torch.empty((wl.grid.n_total, 64, 4), device="cuda")
    sg.compute_integral_field(wl.grid, wl.phi, field)
    out = torch.empty((pos.shape[0], 4), device="cuda")
    sg.probe_integral_field(wl.grid, field, wl.pos, out)
    torch.cuda.synchronize()

    # the field at every activated point
    ref = oracle.integral_field(run.N, run.h, run.B, run.tab, run.active, run.phi)
    f = field[:, torch.from_numpy(_blocked()).cuda(), :].double().cpu().numpy()      # [P+2][64 local][4]
    pts = wl.points                                                                  # [P][64] dense index
    got = f[2:].reshape(-1, 4)
    want = ref[:, pts.ravel()].T
    assert np.max(np.abs(got[:, 0] - want[:, 0])) <= 1e-5
    assert np.max(np.abs(got[:, 1:] - want[:, 1:])) <= 1e-5 * G0
    # the one-sided far-field rows
    c = oracle.c_full()
    assert np.all(f[0] == 0.0)
    assert np.all(f[1, :, 1:] == 0.0) and np.allclose(f[1, :, 0], c, rtol=1e-7)
    # both saturated and cut points occur, inner packages included
    assert (want[:, 0] < 1e-6).mean() > 0.01 and (np.abs(want[:, 0] - c) < 1e-6).mean() > 0.1
    assert ((want[:, 0] > 0.05) & (want[:, 0] < c - 0.05)).mean() > 0.05

    # the probe: interpolation of the oracle field under the same rules
    pr = oracle.probe_field(run.N, run.h, run.tab.cell_pkg, ref, pos.astype(np.float64))
    gp = out.double().cpu().numpy()
    assert np.max(np.abs(gp[:, 0] - pr[:, 0])) <= 2e-5
    assert np.max(np.abs(gp[:, 1:] - pr[:, 1:])) <= 2e-5 * G0
    # particles whose home cell is far field read its constants
    M = N // 4
    cc = np.clip(np.floor(pos.astype(np.float64) * M), 0, M - 1).astype(np.int64)
    home = run.tab.cell_pkg[cc[:, 0] + M * (cc[:, 1] + M * cc[:, 2])]
    assert (home < 2).sum() > 100 and (home >= 2).sum() > 1000
    assert np.all(gp[home == 0] == 0.0)
    # (the eight FP32 weights of a blend of one constant sum to 1 within rounding)
    assert np.allclose(gp[home == 1, 0], c, rtol=1e-6, atol=0) and np.all(gp[home == 1, 1:] == 0.0)


def test_integral_field_rejects_bad_arguments(sg):
    cfg = synth.config_c1()
    from paper_2512_11473_amd import workload
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    with pytest.raises(ValueError):
        sg.compute_integral_field(wl.grid, wl.phi, torch.empty((wl.grid.n_total, 64, 3), device="cuda"))
    with pytest.raises(TypeError):
        sg.probe_integral_field(wl.grid, torch.empty((wl.grid.n_total, 64, 4), device="cuda"),
                                torch.zeros((3, 3), dtype=torch.float64, device="cuda"),
                                torch.empty((3, 4), device="cuda"))
    # no particles: nothing to do
    sg.probe_integral_field(wl.grid, torch.empty((wl.grid.n_total, 64, 4), device="cuda"),
                            torch.empty((0, 3), device="cuda"), torch.empty((0, 4), device="cuda"))
