"""Benchmark of the narrow-band sparse-grid hot path on one MI355X.

Workload (extruded triangular prism, edges 0.6, extrusion 0.8, 512^3 data
points, 4^3 packages within about two package widths of the surface, phi0 =
SDF * (1 + 0.05 u), 100 reinitialisation iterations, central-difference
gradient, 1e7 particles jittered N(0, 0.5h) about the surface, plain
near-surface integrals on every core point).

One step = one pass of the whole hot path over the resident inputs:
package build from the coarse distances, phi reset from phi0 (device copy),
n_iter reinitialisation sweeps, gradient, probe, integrals.  Inputs are
generated once, uploaded, and resident in HBM before timing starts.

Prints one JSON line.  `value` = package-cell updates (64 P n_iter per step)
per second of whole-step time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
REINIT_BYTES_PER_UPDATE = 8.375      # read + write one FP32 value, plus 6 face ids / 64 points
GRAD_BYTES_PER_POINT = 16.375        # read phi, write 3 components, face ids
PROBE_BYTES_PER_PARTICLE = 28.0      # 12 B position in, 16 B value + normal out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-iter", type=int, default=100)
    ap.add_argument("--particles", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8)
    return ap.parse_args()


def cpu_baseline(cfg, n_iter_sample):
    """The oracle (FP64, dense grid, OpenMP) timed on the host on a bounded
    sample of the workload: `n_iter_sample` reinitialisation sweeps over the
    full band, then updates/s."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    run = oracle.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    dense = oracle.dense_state(run.tab, run.active, run.phi0, run.B)
    setup_s = time.perf_counter() - t0
    oracle.reinit(run.N, run.h, run.B, run.active, dense, 1)       # warm-up
    t0 = time.perf_counter()
    oracle.reinit(run.N, run.h, run.B, run.active, dense, n_iter_sample)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(run.active) * n_iter_sample / dt, "unit": "package-cell updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{n_iter_sample} FP64 reinitialisation sweeps over the full prism512 band "
                      f"({len(run.active)} points, {dt:.1f} s; setup {setup_s:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path has no multi-GPU mode",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2512_11473_amd as sg
    import synth
    from paper_2512_11473_amd import workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = synth.config_c2()
    cfg["n_iter"] = args.n_iter
    t0 = time.perf_counter()
    pos = synth.particles_for(cfg, args.particles)
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    setup_s = time.perf_counter() - t0
    P = wl.grid.n_packages
    n_core = wl.grid.n_core
    integ = torch.empty((4, n_core * 64), device="cuda")
    stream = torch.cuda.current_stream()

    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(2)] for k in
          ("build", "reinit", "grad", "probe", "integ")}
    acc = {k: 0.0 for k in ev}

    def step(record):
        def mark(k, i):
            if record:
                ev[k][i].record(stream)
        mark("build", 0)
        g = sg.build_packages(wl.coarse, wl.h)
        mark("build", 1)
        wl.phi.copy_(wl.phi0)
        mark("reinit", 0)
        sg.reinitialize(g, wl.phi, wl.scratch, cfg["n_iter"])
        mark("reinit", 1)
        mark("grad", 0)
        sg.compute_gradient(g, wl.phi, wl.grad)
        mark("grad", 1)
        mark("probe", 0)
        sg.probe_particles(g, wl.phi, wl.grad, wl.pos, wl.phi_p, wl.nrm_p)
        mark("probe", 1)
        mark("integ", 0)
        sg.compute_near_surface_integrals(g, wl.phi, integ)
        mark("integ", 1)
        return g

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    grids = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        grids.append(step(True))
        torch.cuda.synchronize()
        for k in ev:
            acc[k] += ev[k][0].elapsed_time(ev[k][1])
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    for g in grids:
        g.destroy()

    K = args.steps
    ms_step = 1e3 * total_s / K
    upd_step = 64 * P * cfg["n_iter"]
    reinit_ms = acc["reinit"] / K
    sweep_ms = reinit_ms / cfg["n_iter"]
    achieved = REINIT_BYTES_PER_UPDATE * 64 * P / (sweep_ms * 1e-3) / 1e9
    n_pts = 64 * (P + 2)
    rec = {
        "metric": "package-cell updates/s (reinit), probes/s; learned vs plain integral @1e-3",
        "value": upd_step / (ms_step * 1e-3),
        "unit": "package-cell updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "prism512: extruded triangular prism, 512^3, 100 reinit iterations, "
                               "gradient, 1e7 jittered particles, plain integrals",
                   "N": cfg["N"], "n_packages": P, "n_core": n_core, "n_iter": cfg["n_iter"],
                   "particles": int(wl.pos.shape[0])},
        "breakdown_ms": {k: acc[k] / K for k in acc},
        "reinit_updates_per_s": upd_step / (reinit_ms * 1e-3),
        "probes_per_s": wl.pos.shape[0] / (acc["probe"] / K * 1e-3),
        "gradient_points_per_s": n_pts / (acc["grad"] / K * 1e-3),
        "integral_cells_per_s": n_core * 64 / (acc["integ"] / K * 1e-3),
        "roofline": {"bound": "hbm", "kernel": "reinit sweep", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": sweep_ms * 1e3,
                     "bytes_per_launch": REINIT_BYTES_PER_UPDATE * 64 * P},
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(cfg, args.cpu_iters)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
