"""Training and evaluation of the surrogate network for the near-surface
integrals.  The data come from the method itself: seeded random unions are
activated, reinitialised and integrated with the plain kernel; the network
inputs (windows of phi / h) and the saturation flags come from the library's
gather kernel.  Training steps, inference and the gated fallback run in the
library's kernels; this module only drives them and keeps statistics.

Recipe: shapes from the random-union generator at 128^3 and 256^3, 10%
multiplicative noise, 20 reinitialisation iterations, non-saturated core
points only; loss = sum_o (y_o - t_o)^2 / sigma_o^2 (targets standardised by
their training-set spread); Adam with a cosine learning rate from 1e-3 to
1e-5; Kaiming-uniform initialisation scaled by the input spread.  The gate
threshold is the 99.9th percentile of the training windows' non-planarity.
The benchmark trains 300 epochs of 2048-sample batches over 2e6 points, the
best of the step counts and batch sizes tried (held-out mean error 2.5e-3).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

import synth

from . import Mlp, compute_near_surface_integrals, gather_windows, reinitialize
from . import workload

C_FULL = 0.9805454147235685     # K_W of a fully outside neighbourhood
G0 = 0.865663036                # h |K_grad| of a half-space through the query point


@dataclass
class Dataset:
    x: torch.Tensor      # [n, 216] float32 windows of phi / h
    t: torch.Tensor      # [n, 4] plain integrals (K_W, h K_grad)
    shapes: int
    seconds: float


def generate(n_shapes: int, seed: int, max_cells: int, resolutions=(128, 256), n_iter: int = 20,
             noise_amp: float = 0.1) -> Dataset:
    """Non-saturated core points of `n_shapes` seeded shapes, at most
    `max_cells` in total (spread evenly over the shapes)."""
    t0 = time.perf_counter()
    specs = synth.batch_shapes(n_shapes, seed, resolutions=resolutions)
    per = max(1, max_cells // n_shapes)
    xs, ts = [], []
    gen = torch.Generator(device="cpu").manual_seed(seed)
    for s in specs:
        wl = workload.setup(s["shape"], s["N"], noise_amp, s["noise_seed"])
        reinitialize(wl.grid, wl.phi, wl.scratch, n_iter)
        n = wl.grid.n_core * 64
        if n == 0:
            continue
        out = torch.empty((4, n), device="cuda")
        compute_near_surface_integrals(wl.grid, wl.phi, out)
        x = torch.empty((n, 216), device="cuda")
        un = torch.empty(n, dtype=torch.uint8, device="cuda")
        gather_windows(wl.grid, wl.phi, x, un)
        idx = torch.nonzero(un, as_tuple=False).ravel()
        if idx.numel() > per:
            pick = torch.randperm(idx.numel(), generator=gen)[:per].to(idx.device)
            idx = idx[pick]
        xs.append(x[idx])
        ts.append(out[:, idx].t().contiguous())
        wl.grid.destroy()
        del wl, x, out, un
    x = torch.cat(xs).contiguous()
    t = torch.cat(ts).contiguous()
    torch.cuda.synchronize()
    return Dataset(x, t, len(specs), time.perf_counter() - t0)


def nonplanarity(x: torch.Tensor) -> torch.Tensor:
    """Mean squared residual of each window after its least-squares affine fit
    (the affine basis 1, ox, oy, oz is orthogonal on the 6^3 window)."""
    o = torch.arange(6, device=x.device, dtype=torch.float32) - 2.5
    ox = o.repeat(36)
    oy = o.repeat_interleave(6).repeat(6)
    oz = o.repeat_interleave(36)
    c0 = x.mean(dim=1, keepdim=True)
    cx = (x * ox).sum(dim=1, keepdim=True) / 630.0
    cy = (x * oy).sum(dim=1, keepdim=True) / 630.0
    cz = (x * oz).sum(dim=1, keepdim=True) / 630.0
    r = x - c0 - cx * ox - cy * oy - cz * oz
    return (r * r).mean(dim=1)


def init_params(seed: int, x_scale: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in, s in [(128, 216, 1.0 / max(x_scale, 1e-6)), (128, 128, 1.0), (4, 128, 0.1)]:
        lim = math.sqrt(6.0 / fan_in) * s
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def relative_error(y: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Per-point error max(|dK_W| / C, h |dK_grad|_2 / G0)."""
    ew = (y[:, 0] - t[:, 0]).abs() / C_FULL
    eg = torch.linalg.norm(y[:, 1:] - t[:, 1:], dim=1) / G0
    return torch.maximum(ew, eg)


def error_stats(e: torch.Tensor) -> Dict[str, float]:
    e = e.double()
    return {"mean": float(e.mean()), "p99": float(torch.quantile(e[:1_000_000], 0.99)),
            "max": float(e.max()), "n": int(e.numel())}


@dataclass
class TrainResult:
    model: Mlp
    losses: List[float]
    seconds: float
    steps: int
    tau: float
    sigma: List[float]
    x_scale: float


def train(data: Dataset, epochs: int, batch: int = 4096, lr0: float = 1e-3, lr1: float = 1e-5,
          seed: int = 0, log=None) -> TrainResult:
    n = data.x.shape[0]
    sigma = data.t.std(dim=0).clamp_min(1e-6)
    mean = data.t.mean(dim=0)
    lw = (1.0 / sigma ** 2).cpu().numpy().astype(np.float32)
    x_scale = float(data.x.std())
    w = init_params(seed, x_scale)
    w[-4:] = mean.cpu().numpy()              # output bias starts at the target mean
    model = Mlp(w)
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    loss = torch.zeros(1, device="cuda")
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        ep_loss = torch.zeros(1, device="cuda", dtype=torch.float64)
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            xb = data.x[idx]
            tb = data.t[idx]
            lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * step / total))
            model.train_step(xb, tb, lw, lr, loss)
            ep_loss += loss.double()
            step += 1
        losses.append(float(ep_loss.item()) / (steps_per_epoch * batch * 4))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean standardised squared error {losses[-1]:.3e}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    npl = nonplanarity(data.x[:min(n, 2_000_000)])
    tau = float(torch.quantile(npl[:1_000_000].double(), 0.999))
    model.set_gate(tau)
    return TrainResult(model, losses, secs, step, tau, sigma.cpu().tolist(), x_scale)


def evaluate(model: Mlp, data: Dataset, tau: Optional[float] = None) -> Dict:
    """Ungated and gated errors on held-out points: the gate keeps a point when
    its non-planarity is <= tau and K_W is in range; other points take the
    plain value (error 0)."""
    n = data.x.shape[0]
    y = torch.empty((n, 4), device="cuda")
    model.forward(data.x, y)
    e = relative_error(y, data.t)
    res = {"ungated": error_stats(e)}
    if tau is not None:
        keep = (nonplanarity(data.x) <= tau) & (y[:, 0] >= -0.05) & (y[:, 0] <= 1.05)
        eg = torch.where(keep, e, torch.zeros_like(e))
        res["gated"] = error_stats(eg)
        res["fallback_fraction"] = float(1.0 - keep.float().mean())
    return res
