"""The surrogate network's HIP kernels against the FP64 oracle (GPU).

The kernels compute in BF16 with FP32 accumulation, so the oracle is run on
the same BF16-rounded weights and the tolerances are BF16 bounds: activations
carry a relative rounding error of 2^-9 per layer, which bounds the relative
error of outputs and gradients at about 1e-2.
"""
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
    rng = np.random.default_rng(2)
    for B in (1, 15, 64, 333):
        x = (rng.standard_normal((B, 216)) * 2.0).astype(np.float32)
        y = torch.empty((B, 4), device="cuda")
        model.forward(torch.from_numpy(x).cuda(), y)
        ref = oracle.mlp_forward(quantised(w), x.astype(np.float64))
        got = y.double().cpu().numpy()
        scale = max(1.0, np.sqrt((ref ** 2).mean()))
        assert np.max(np.abs(got - ref)) <= 2e-2 * scale, (B, np.max(np.abs(got - ref)))


def test_backward_matches_oracle_and_is_deterministic(sg):
    w = init_params(3)
    model = sg.Mlp(w)
    rng = np.random.default_rng(4)
    B = 300
    x = (rng.standard_normal((B, 216)) * 2.0).astype(np.float32)
    dy = rng.standard_normal((B, 4)).astype(np.float32)
    g = torch.empty(sg.MLP_N_PARAMS, device="cuda")
    xd, dyd = torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda()
    model.backward(xd, dyd, g)
    g1 = g.clone()
    model.backward(xd, dyd, g)
    assert torch.equal(g, g1)
    ref = oracle.mlp_backward(quantised(w), x.astype(np.float64), dy.astype(np.float64))
    got = g.double().cpu().numpy()
    for name, lo, hi in [("W1", 0, 27648), ("b1", 27648, 27776), ("W2", 27776, 44160), ("b2", 44160, 44288),
                         ("W3", 44288, 44800), ("b3", 44800, 44804)]:
        err = np.linalg.norm(got[lo:hi] - ref[lo:hi]) / np.linalg.norm(ref[lo:hi])
        assert err < 2e-2, (name, err)


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
    assert torch.max(torch.abs(out - plain)).item() <= 1e-6
    # tau = inf and a wide range: every non-saturated point takes the network
    model.set_gate(3.0e38, -1e30, 1e30)
    sg.compute_near_surface_integrals(wl.grid, wl.phi, out, model=model, n_fallback=nf)
    y = torch.empty((n, 4), device="cuda")
    model.forward(x, y)
    torch.cuda.synchronize()
    assert int(nf.item()) == 0
    m = un.bool()
    assert torch.equal(out[:, m], y[m].t().contiguous())
    assert torch.max(torch.abs(out[:, ~m] - plain[:, ~m])).item() <= 1e-6


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
