"""The surrogate network's HIP kernels against the FP64 oracle (GPU).

The kernels compute in BF16 with FP32 accumulation, so the oracle is run on
the same BF16-rounded weights and each output and gradient element is held
to K_SIGMA standard deviations of the kernels' rounding error, propagated
through the network in tests/mlp_bounds.py (about 5 % of a typical element;
a copied neighbouring entry lies far outside).  Adam runs in FP32 against
the oracle's FP64 update; the gate's decisions are checked against an FP64
least-squares plane fit of every window.
"""
import numpy as np
import pytest

import mlp_bounds as mb
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
    return sg


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even)."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def init_params(seed):
    """Kaiming-uniform weights (fan-in), small biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in [(128, 216), (128, 128), (4, 128)]:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(rng.uniform(-0.1, 0.1, fan_out))
    return np.concatenate(parts).astype(np.float32)


def quantised(w):
    """The weights as the kernels see them: BF16 matrices, FP32 biases."""
    q = w.astype(np.float64).copy()
    for lo, hi in [(0, 27648), (27776, 44160), (44288, 44800)]:
        q[lo:hi] = bf16_round(w[lo:hi])
    return q


def test_forward_matches_oracle(sg):
    w = init_params(1)
    model = sg.Mlp(w)
    q = quantised(w)
    rng = np.random.default_rng(2)
    for B in (1, 15, 64, 333):
        x = (rng.standard_normal((B, 216)) * 2.0).astype(np.float32)
        y = torch.empty((B, 4), device="cuda")
        model.forward(torch.from_numpy(x).cuda(), y)
        f = mb.forward_scales(q, x.astype(np.float64))
        ref = oracle.mlp_forward(q, x.astype(np.float64))
        got = y.double().cpu().numpy()
        assert np.allclose(ref, f["y"], rtol=1e-12, atol=1e-12)     # the scales' activations are the oracle's
        err = np.abs(got - ref) / np.sqrt(f["v_y"])
        assert err.max() <= mb.K_SIGMA, (B, err.max())


@pytest.mark.parametrize("B,seed", [(64, 3), (300, 13)])
def test_backward_matches_oracle_elementwise(sg, B, seed):
    w = init_params(seed)
    model = sg.Mlp(w)
    rng = np.random.default_rng(seed + 1)
    x = (rng.standard_normal((B, 216)) * 2.0).astype(np.float32)
    dy = rng.standard_normal((B, 4)).astype(np.float32)
    g = torch.empty(sg.MLP_N_PARAMS, device="cuda")
    xd, dyd = torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda()
    model.backward(xd, dyd, g)
    g1 = g.clone()
    model.backward(xd, dyd, g)
    assert torch.equal(g, g1)                                      # fixed reduction order
    q = quantised(w)
    ref = oracle.mlp_backward(q, x.astype(np.float64), dy.astype(np.float64))
    sd = mb.backward_scales(q, w.astype(np.float64), x.astype(np.float64), dy.astype(np.float64))
    got = g.double().cpu().numpy()
    z = np.abs(got - ref) / sd
    for name, (lo, hi) in mb._SLICES.items():
        worst = int(np.argmax(z[lo:hi])) + lo
        assert z[lo:hi].max() <= mb.K_SIGMA, (name, worst, got[worst], ref[worst], sd[worst])
    # the scale is a few per cent of a typical element, so a wrong entry shows
    assert np.median(mb.K_SIGMA * sd[:27648] / np.abs(ref[:27648])) < 0.1


def test_apply_gradient_five_adam_steps_match_oracle(sg):
    """Five Adam steps from given gradients of changing sign and scale: the
    FP32 moments and parameters against the oracle's FP64 update."""
    w = init_params(21)
    model = sg.Mlp(w)
    rng = np.random.default_rng(22)
    n = sg.MLP_N_PARAMS
    lr = 1e-3
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))    # the kernel's decay rates
    w_ref, m_ref, v_ref = w.astype(np.float64), np.zeros(n), np.zeros(n)
    grads = []
    for t in range(1, 6):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
        grads.append(g.astype(np.float64))
        model.apply_gradient(torch.from_numpy(g).cuda(), lr)
        oracle.adam(w_ref, g.astype(np.float64), m_ref, v_ref, t, lr, beta1=b1, beta2=b2)
        wg, mg, vg, step = model.state()
        assert step == t
        G = np.abs(np.array(grads))
        k = np.arange(t - 1, -1, -1)[:, None]
        m_mag = (1 - b1) * (b1 ** k * G).sum(0)             # sum of |terms| of m_t
        v_mag = (1 - b2) * (b2 ** k * G * G).sum(0)
        assert np.all(np.abs(mg - m_ref) <= 1e-6 * m_mag + 1e-30), t
        assert np.all(np.abs(vg - v_ref) <= 1e-6 * v_mag + 1e-38), t
        # each step adds at most half an ulp of w (FP32 storage) and a relative
        # 1e-6 of its size, lr |m_hat| / (sqrt(v_hat) + eps) <= lr (1 - b1) /
        # sqrt(1 - b2) (Kingma and Ba, Sec. 2.1)
        ulp = np.spacing(np.abs(w_ref).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(wg - w_ref) <= t * ulp + 1e-6 * t * lr * (1 - b1) / np.sqrt(1 - b2)), t


def _windows_and_outputs(sg, model, tau, kw_lo, kw_hi):
    cfg, wl = _sphere_grid(sg)
    n = wl.grid.n_core * 64
    plain = torch.empty((4, n), device="cuda")
    sg.compute_near_surface_integrals(wl.grid, wl.phi, plain)
    x = torch.empty((n, 216), device="cuda")
    un = torch.empty(n, dtype=torch.uint8, device="cuda")
    sg.gather_windows(wl.grid, wl.phi, x, un)
    y = torch.empty((n, 4), device="cuda")
    model.forward(x, y)
    model.set_gate(tau, kw_lo, kw_hi)
    out = torch.empty_like(plain)
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    sg.compute_near_surface_integrals(wl.grid, wl.phi, out, model=model, n_fallback=nf)
    torch.cuda.synchronize()
    un = un.cpu().numpy().astype(bool)
    y, out, plain = y.cpu().numpy(), out.cpu().numpy().T, plain.cpu().numpy().T
    learned = np.all(out == y, axis=1)
    fell = ~learned & np.all(out == plain, axis=1)
    assert np.all(learned | fell)                  # every point took one of the two values, bit for bit
    assert np.all(fell[~un])                      # saturated points: the exact (plain) value
    assert int(nf.item()) == int((fell & un).sum())
    return x.cpu().numpy().astype(np.float64), un, y, fell


def test_gate_nonplanarity_decisions_match_fp64_fit(sg):
    """At thresholds across the distribution, a non-saturated point falls back
    exactly when the FP64 mean squared residual of its window's least-squares
    plane fit exceeds tau, except within the FP32 rounding of the kernel's
    explicit residual sum around tau."""
    model = sg.Mlp(init_params(9))
    x, un, y, fell = _windows_and_outputs(sg, model, 3.0e38, -1e30, 1e30)
    res = mb.nonplanarity_f64(x[un])
    slack = mb.nonplanarity_f32_bound(x[un])
    assert not fell[un].any()
    for qtl in (0.1, 0.5, 0.9, 0.999):
        tau = float(np.quantile(res, qtl))
        _, _, _, fell = _windows_and_outputs(sg, model, tau, -1e30, 1e30)
        f = fell[un]
        sure_in, sure_out = res < tau - slack, res > tau + slack
        assert not f[sure_in].any(), (qtl, int(f[sure_in].sum()))
        assert f[sure_out].all(), (qtl, int((~f[sure_out]).sum()))
        assert (sure_in | sure_out).mean() > 0.99                  # the rounding band is narrow
        assert abs(f.mean() - (1.0 - qtl)) < 0.02


def test_gate_kw_range_decisions(sg):
    """With the residual test open, a non-saturated point falls back exactly
    when the network's K_W lies outside [kw_lo, kw_hi] (the same FP32 value
    in both places)."""
    model = sg.Mlp(init_params(9))
    _, un, y, _ = _windows_and_outputs(sg, model, 3.0e38, -1e30, 1e30)
    lo, hi = (float(v) for v in np.quantile(y[un, 0], [0.2, 0.7]))
    _, un, y, fell = _windows_and_outputs(sg, model, 3.0e38, lo, hi)
    expect = un & ((y[:, 0] < np.float32(lo)) | (y[:, 0] > np.float32(hi)))
    assert np.array_equal(fell & un, expect)


def test_adam_first_step(sg):
    w = init_params(5)
    model = sg.Mlp(w)
    rng = np.random.default_rng(6)
    B = 256
    x = (rng.standard_normal((B, 216)) * 2.0).astype(np.float32)
    t = rng.standard_normal((B, 4)).astype(np.float32)
    lw = np.array([1.0, 2.0, 0.5, 1.5], dtype=np.float32)
    loss = torch.zeros(1, device="cuda")
    lr = 1e-3
    model.train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), lw, lr, loss)
    w1, m1, v1, step = model.state()
    assert step == 1
    # oracle: gradient of sum_o w_o (y - t)^2 / B on the same quantised weights
    q = quantised(w)
    y = oracle.mlp_forward(q, x.astype(np.float64))
    dy = 2.0 * lw[None, :] * (y - t) / B
    g = oracle.mlp_backward(q, x.astype(np.float64), dy)
    ref_loss = float((lw[None, :] * (y - t) ** 2).sum())
    assert abs(loss.item() - ref_loss) <= 2e-2 * ref_loss
    # the first bias-corrected Adam step moves every parameter by lr * sign(g)
    step_gpu = w.astype(np.float64) - w1.astype(np.float64)
    robust = np.abs(g) > 1e-2 * np.abs(g).max()
    agree = np.isclose(step_gpu[robust], lr * np.sign(g[robust]), rtol=1e-3, atol=1e-7)
    assert agree.mean() > 0.99
    assert np.all(np.abs(step_gpu) <= lr * 1.001 + 1e-7)
    # moments: m = 0.1 g, v = 0.001 g^2 (within BF16 bounds of g)
    assert np.linalg.norm(m1 - 0.1 * g) <= 2e-2 * np.linalg.norm(0.1 * g)


def test_training_reduces_loss(sg):
    # fit a fixed random linear map of the inputs (learnable by the network)
    rng = np.random.default_rng(7)
    B = 4096
    x = (rng.standard_normal((B, 216)) * 1.5).astype(np.float32)
    A = rng.standard_normal((216, 4)) / np.sqrt(216)
    t = np.tanh(x @ A).astype(np.float32)
    model = sg.Mlp(init_params(8))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss = torch.zeros(1, device="cuda")
    losses = []
    for it in range(150):
        model.train_step(xd, td, [1, 1, 1, 1], 2e-3, loss)
        losses.append(loss.item() / B)
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])


def _sphere_grid(sg, n_iter=5):
    from paper_2512_11473_amd import workload
    cfg = synth.config_c1()
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
    return cfg, wl


def test_gather_windows_match_oracle(sg):
    cfg, wl = _sphere_grid(sg)
    n = wl.grid.n_core * 64
    x = torch.empty((n, 216), device="cuda")
    un = torch.empty(n, dtype=torch.uint8, device="cuda")
    sg.gather_windows(wl.grid, wl.phi, x, un)
    core = wl.grid.tables()["core_list"].cpu().numpy().astype(np.int64)
    pts = wl.points[core - 2].ravel()
    # dense state from the GPU field: windows are a pure re-indexing of phi
    N, h = wl.N, wl.h
    dense = np.full(N ** 3, np.nan)
    dense[wl.points.ravel()] = wl.phi[2:].double().cpu().numpy().ravel()
    run = oracle.setup(cfg["shape"], N, cfg["noise_amp"], cfg["noise_seed"])
    far = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    dense = np.where(np.isnan(dense), far, dense)
    ref = oracle.windows(N, h, 16 * h, dense, pts)
    assert np.array_equal(x.double().cpu().numpy(), ref)
    u = un.cpu().numpy()
    assert 0.2 < u.mean() < 0.9


def test_learned_integrals_gate_extremes(sg):
    cfg, wl = _sphere_grid(sg)
    n = wl.grid.n_core * 64
    plain = torch.empty((4, n), device="cuda")
    sg.compute_near_surface_integrals(wl.grid, wl.phi, plain)
    un = torch.empty(n, dtype=torch.uint8, device="cuda")
    x = torch.empty((n, 216), device="cuda")
    sg.gather_windows(wl.grid, wl.phi, x, un)
    model = sg.Mlp(init_params(9))
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty_like(plain)
    # tau = 0: every non-saturated point falls back to the plain integral
    model.set_gate(0.0)
    sg.compute_near_surface_integrals(wl.grid, wl.phi, out, model=model, n_fallback=nf)
    torch.cuda.synchronize()
    assert int(nf.item()) == int(un.sum().item())
    assert torch.equal(out, plain)          # the fallback and the saturated sums are the plain kernels' bits
    # tau = inf and a wide range: every non-saturated point takes the network
    model.set_gate(3.0e38, -1e30, 1e30)
    sg.compute_near_surface_integrals(wl.grid, wl.phi, out, model=model, n_fallback=nf)
    y = torch.empty((n, 4), device="cuda")
    model.forward(x, y)
    torch.cuda.synchronize()
    assert int(nf.item()) == 0
    m = un.bool()
    assert torch.equal(out[:, m], y[m].t().contiguous())
    assert torch.equal(out[:, ~m], plain[:, ~m])


def test_trained_surrogate_against_plain(sg):
    """What the trained network gives over the method without it: trained by
    the library's kernels on points of seeded shapes, it reproduces the plain
    integrals of held-out shapes far better than before training, and the
    gated learned path on a grid stays within the fallback contract.  The
    timing of both paths is recorded (the plain kernel is the faster one)."""
    from paper_2512_11473_amd import surrogate, workload
    tr = surrogate.generate(16, 303, 200_000, resolutions=(64, 128))
    ho = surrogate.generate(8, 404, 100_000, resolutions=(64, 128))
    assert tr.x.shape[0] > 100_000 and ho.x.shape[0] > 50_000
    res = surrogate.train(tr, epochs=30, batch=2048)
    before = surrogate.evaluate(sg.Mlp(surrogate.init_params(0, float(tr.x.std()))), ho)["ungated"]["mean"]
    after = surrogate.evaluate(res.model, ho, res.tau)
    assert after["ungated"]["mean"] < before / 10
    assert after["ungated"]["mean"] < 2e-2
    assert after["fallback_fraction"] < 0.05
    # on a grid: learned + fallback against plain
    cfg = synth.config_c1()
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    sg.reinitialize(wl.grid, wl.phi, wl.scratch, 20)
    n = wl.grid.n_core * 64
    plain = torch.empty((4, n), device="cuda")
    learned = torch.empty_like(plain)
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    sg.compute_near_surface_integrals(wl.grid, wl.phi, plain)
    e[1].record()
    sg.compute_near_surface_integrals(wl.grid, wl.phi, learned, model=res.model, n_fallback=nf)
    e[2].record()
    torch.cuda.synchronize()
    err = surrogate.relative_error(learned.t(), plain.t())
    assert float(err.mean()) < 2e-2
    print(f"\nsurrogate: held-out mean error {before:.3e} -> {after['ungated']['mean']:.3e}; "
          f"grid mean error {float(err.mean()):.3e}, fallback {int(nf.item())} of {n}; "
          f"plain {e[0].elapsed_time(e[1]):.3f} ms, learned {e[1].elapsed_time(e[2]):.3f} ms")


def test_checkpoint_resume_is_bit_identical(sg):
    """Training resumed from a checkpoint (master weights, Adam moments, step
    count) continues exactly as the uninterrupted run: the weight-gradient
    reduction runs in a fixed order, so the same inputs give the same bits."""
    rng = np.random.default_rng(11)
    B = 1024
    batches = [(torch.from_numpy((rng.standard_normal((B, 216)) * 1.5).astype(np.float32)).cuda(),
                torch.from_numpy(rng.standard_normal((B, 4)).astype(np.float32)).cuda()) for _ in range(6)]
    loss = torch.zeros(1, device="cuda")
    lw = [1.0, 0.5, 2.0, 1.0]
    a = sg.Mlp(init_params(12))
    for x, t in batches:
        a.train_step(x, t, lw, 1e-3, loss)
    b = sg.Mlp(init_params(12))
    for x, t in batches[:3]:
        b.train_step(x, t, lw, 1e-3, loss)
    w, m, v, step = b.state()
    c = sg.Mlp(w)
    c.set_state(m, v, step)
    for x, t in batches[3:]:
        c.train_step(x, t, lw, 1e-3, loss)
    wa, ma, va, sa = a.state()
    wc, mc, vc, sc = c.state()
    assert sa == sc == 6
    assert np.array_equal(wa, wc) and np.array_equal(ma, mc) and np.array_equal(va, vc)
