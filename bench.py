"""Benchmark of the narrow-band sparse-grid hot path on one MI355X.

Default workload (torus2048): torus R = 0.35, r = 0.1 whose surface is
displaced by 0.02 x a sum of 8 seeded sinusoidal modes, at 2048^3 data points
(narrow band only: 4^3 packages within about two package widths of the
surface), phi0 = SDF * (1 + 0.05 u); 100 reinitialisation iterations, the
central-difference gradient, 5e7 particles jittered N(0, 0.5h) about the
surface (sorted by home cell, then probed), and the near-surface integrals
of every core point by the learned surrogate with its residual gate and
plain fallback.

One step = one pass of the whole hot path over resident inputs: package
build from the coarse distances, phi reset from phi0 (device copy), 100
reinitialisation sweeps, packed gradient, sort of the particles by home
cell (Morton order) and the probe of the sorted particles, learned
integrals with gate and fallback.  Inputs are generated once and resident in HBM before timing
starts; the surrogate is trained before timing (by the library's training
kernels, on points of 256 other seeded shapes).

`value` = package-cell updates (64 P n_iter per step) per second of
whole-step time.  The plain integrals (direct and factorised) are timed
beside the step, with the learned error against them; the probe in generated
particle order, and the oracle's CPU baseline, are added to the same JSON
line.

Other workloads: --workload prism512 (extruded triangular prism, edges 0.6,
extrusion 0.8, at 512^3: the same step with 1e7 particles), batch64 (64
random unions, one persistent launch per iteration, graph replay, autotuned
configuration) and shell1024 (the paper's timing test).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
REINIT_BYTES_PER_UPDATE = 8.375      # read + write one FP32 value, plus 6 face ids / 64 points
PROBE_BYTES_PER_PARTICLE = 28.0      # 12 B position in, 16 B value + normal out
# the sources the sweep and stencil kernels are compiled from: a counter
# summary counts only while they are unchanged
SWEEP_SRCS = [os.path.join(ROOT, "paper_2512_11473_amd", "csrc", f) for f in ("sweep.hip", "common.hpp", "upwind.hpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="torus2048", choices=["prism512", "torus2048", "batch64", "shell1024"])
    ap.add_argument("--n-iter", type=int, default=None)
    ap.add_argument("--sweep", default="auto",
                    help="sweep configuration 'variant,groups', or 'auto' to autotune it on the grid (default)")
    ap.add_argument("--particles", type=int, default=None, help="default: the workload's count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="no surrogate: the step takes the plain integrals (factorised) instead")
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle sweeps per CPU-baseline pass (default: the workload's iteration count)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum oracle sweeping time of the CPU baseline")
    ap.add_argument("--train-cells", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--train-batch", type=int, default=2048)
    ap.add_argument("--overlap", action="store_true",
                    help="run the integrals on a second stream beside the gradient and the probe (a shorter step "
                         "at torus2048, a slightly slower sweep at prism512)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration under rocprofv3)")
    return ap.parse_args()


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(summary: str, key: str):
    """HBM bytes per launch of one kernel configuration (`key`) from a committed
    rocprofv3 counter summary under profiles/, when the summary was taken on
    the current sweep sources; else None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sweep_sources_sha256_16:\s*(\w+)", text)
    t = re.search(r"calibrated_bytes_per_launch\[" + re.escape(key) + r"\]:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != sweep_source_hash():
        return None
    return float(t.group(1))


# 100^3-coarse-cell crops around the top of the torus tube at four angles:
# the oracle's samples of the 2048^3 band
TORUS_CROPS = [(385, 206, 257), (206, 385, 257), (26, 206, 257), (206, 26, 257)]
TORUS_CROP_EXTENT = 100


def _omp():
    """The OpenMP runtime the oracle's library uses (libgomp, already loaded)."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = ctypes.c_int
    gomp.omp_set_num_threads.argtypes = [ctypes.c_int]
    return gomp


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, n_iter, min_seconds=10.0, one_thread_seconds=4.0):
    """The oracle (FP64, dense grid, OpenMP) timed on the host on a bounded
    sample of the workload: passes of `n_iter` reinitialisation sweeps from
    phi0 over the full band (or, at 2048^3 where the dense grid would not fit,
    over crops of it in turn), repeated until `min_seconds` of sweeping with
    every thread the runtime gives it; then the same on one thread for at
    least `one_thread_seconds` (fewer sweeps per pass)."""
    import oracle
    t0 = time.perf_counter()
    if cfg["N"] > 1024:
        runs = [oracle.setup_crop(cfg["shape"], cfg["N"], o, TORUS_CROP_EXTENT, cfg["noise_amp"], cfg["noise_seed"])
                for o in TORUS_CROPS]
        where = f"{len(runs)} crops of {TORUS_CROP_EXTENT}^3 coarse cells of the {cfg['name']} band in turn"
    else:
        runs = [oracle.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])]
        where = f"the full {cfg['name']} band"
    dense = [oracle.dense_state(r.tab, r.active, r.phi0, r.B) for r in runs]
    setup_s = time.perf_counter() - t0
    oracle.reinit(runs[0].N, runs[0].h, runs[0].B, runs[0].active, dense[0], 1)       # warm-up

    def timed(iters, seconds):
        updates, secs, passes = 0, 0.0, 0
        while secs < seconds:
            r, d = runs[passes % len(runs)], dense[passes % len(runs)]
            t1 = time.perf_counter()
            oracle.reinit(r.N, r.h, r.B, r.active, d, iters)
            secs += time.perf_counter() - t1
            updates += len(r.active) * iters
            passes += 1
        return updates / secs, secs, passes

    gomp = _omp()
    threads = gomp.omp_get_max_threads()
    rate, secs, passes = timed(n_iter, min_seconds)
    gomp.omp_set_num_threads(1)
    try:
        one_iters = max(1, n_iter // 10)
        rate1, secs1, passes1 = timed(one_iters, one_thread_seconds)
    finally:
        gomp.omp_set_num_threads(threads)
    pts = sum(len(r.active) for r in runs) // len(runs)
    return {"value": rate, "unit": "package-cell updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread_value": rate1,
            "sample": f"{passes} pass{'es' if passes != 1 else ''} of {n_iter} FP64 reinitialisation sweeps of the "
                      f"oracle over {where} ({pts} points per pass, {secs:.1f} s of sweeping on {threads} threads; "
                      f"one thread: {passes1} passes of {one_iters} sweeps, {secs1:.1f} s; dense-grid setup "
                      f"{setup_s:.1f} s)"}


def train_surrogate(args, log):
    """The surrogate trained by the library's kernels on points of 256 seeded
    random shapes, with a held-out score on points of 128 others."""
    from paper_2512_11473_amd import surrogate
    tr = surrogate.generate(256, 101, args.train_cells)
    ho = surrogate.generate(128, 202, args.train_cells // 2)
    log(f"surrogate data: train {tuple(tr.x.shape)} in {tr.seconds:.1f}s, held-out {tuple(ho.x.shape)}")
    res = surrogate.train(tr, epochs=args.epochs, batch=args.train_batch, log=None)
    log(f"surrogate trained: {res.steps} steps in {res.seconds:.1f}s, final loss {res.losses[-1]:.3e}")
    ev = surrogate.evaluate(res.model, ho, res.tau)
    info = {"heldout": ev,
            "train": {"points": int(tr.x.shape[0]), "shapes": tr.shapes, "epochs": args.epochs,
                      "batch": args.train_batch, "steps": res.steps, "seconds": res.seconds,
                      "final_loss": res.losses[-1], "gate_tau": res.tau}}
    del tr, ho
    return res.model, info


def integrals_report(sg, g, wl, model, log):
    """Learned (gated, with fallback) against both plain forms on the
    benchmark grid's core points after the step: rates and the learned error
    against the plain values."""
    import torch
    from paper_2512_11473_amd import surrogate
    n = g.n_core * 64
    out_p = torch.empty((4, n), device="cuda")
    out_f = torch.empty((4, n), device="cuda")
    vfrac = torch.empty_like(wl.phi)

    def t(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_direct = t(lambda: sg.compute_near_surface_integrals(g, wl.phi, out_p))
    ms_fact = t(lambda: sg.compute_near_surface_integrals_factorised(g, wl.phi, vfrac, out_f))
    same = bool(torch.equal(out_p, out_f))
    del out_f, vfrac
    rec = {"plain_direct_cells_per_s": n / (ms_direct * 1e-3),
           "plain_factorised_cells_per_s": n / (ms_fact * 1e-3),
           "factorised_equals_direct": same}
    if model is not None:
        out_l = torch.empty((4, n), device="cuda")
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        ms_learn = t(lambda: sg.compute_near_surface_integrals(g, wl.phi, out_l, model=model, n_fallback=nf))
        e = surrogate.relative_error(out_l.t(), out_p.t())
        rec.update({"learned_cells_per_s": n / (ms_learn * 1e-3),
                    "learned_over_plain_direct": ms_direct / ms_learn,
                    "learned_over_plain_factorised": ms_fact / ms_learn,
                    "target_rel_error": 1e-3,
                    "bench_grid_error": surrogate.error_stats(e),
                    "bench_grid_fallback_fraction": int(nf.item()) / n})
        log(f"integrals: plain direct {ms_direct:.2f} ms, factorised {ms_fact:.2f} ms, learned {ms_learn:.2f} ms")
    return rec


WORKLOAD_TEXT = {
    "prism512": "prism512: extruded triangular prism (edges 0.6, extrusion 0.8) at 512^3, 5% noise, "
                "100 reinitialisation iterations, gradient, sort and probe of 1e7 jittered particles, "
                "near-surface integrals on all core points",
    "torus2048": "torus2048: torus R=0.35, r=0.1 displaced by 0.02 x 8 seeded modes at 2048^3 (narrow band "
                 "only), 100 reinitialisation iterations, gradient, sort and probe of 5e7 jittered particles, "
                 "near-surface integrals on all core points",
}


def multires_build(sg, synth, cfg, dense_grid, log, levels=2, reps=5):
    """The multi-resolution construction of the same band (Sec. 7): the layer
    at 1/2^levels of the resolution built from its dense distances, then
    `levels` refinements that each evaluate distances only under the previous
    layer's core cells.  The child distances are sampled on the host once
    (they depend only on the core cells); the timed chain runs from device-
    resident inputs, like the step's dense build, and must give its tables."""
    import numpy as np
    import torch
    M = cfg["N"] // 4 >> levels
    d0 = torch.from_numpy(synth.coarse_sdf(cfg["shape"], M)).cuda()
    h0 = 1.0 / (4 * M)
    g = sg.build_packages(d0, h0)
    children = []
    for lv in range(levels):
        t = g.tables()
        cells = t["pkg_cell"].cpu().numpy().view(np.uint32)[t["core_list"].cpu().numpy().astype(np.int64)]
        ch = torch.from_numpy(synth.child_sdf(cfg["shape"], cells.astype(np.int64), M << lv)).cuda()
        children.append(ch)
        g_next = sg.build_packages_refined(g, ch)
        g.destroy()
        g = g_next
    same = g.n_packages == dense_grid.n_packages and all(
        torch.equal(a, b) for a, b in zip(g.tables().values(), dense_grid.tables().values()))
    g.destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = sg.build_packages(d0, h0)
        for ch in children:
            g_next = sg.build_packages_refined(g, ch)
            g.destroy()
            g = g_next
        g.destroy()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    in_bytes = 4 * (M ** 3 + sum(int(c.numel()) for c in children))
    log(f"multi-resolution build: {ms:.2f} ms, tables equal to the dense build: {same}")
    return {"levels": levels + 1, "coarsest_n_coarse": M, "ms": ms, "tables_equal_dense": bool(same),
            "distance_input_bytes": in_bytes, "dense_input_bytes": 4 * (cfg["N"] // 4) ** 3,
            "note": "wall time of the whole chain (each build synchronises once to learn P), measured outside the step"}


def sign_correction(sg, cfg, wl, log):
    """Both steps of the sign correction (Sec. 7.2) on inputs made leaky by
    flipping signs inside eight boxes away from the surface: the coarse step on
    the coarse distances, the refined step on the band's field.  Wall time of
    each call (they synchronise every 16 rounds); the repaired values are
    checked against the unbroken ones."""
    import torch
    M = cfg["N"] // 4
    g = torch.Generator(device="cpu").manual_seed(97)

    def boxes(n_axis):
        lo = torch.randint(0, n_axis - n_axis // 8, (8, 3), generator=g)
        return lo, lo + n_axis // 6

    def in_boxes(i, j, k, lo, hi):
        m = torch.zeros_like(i, dtype=torch.bool)
        for b in range(lo.shape[0]):
            m |= (i >= lo[b, 0]) & (i < hi[b, 0]) & (j >= lo[b, 1]) & (j < hi[b, 1]) & (k >= lo[b, 2]) & (k < hi[b, 2])
        return m

    c = torch.arange(M ** 3, device="cuda")
    lo, hi = boxes(M)
    flip = in_boxes(c % M, (c // M) % M, c // (M * M), lo.cuda(), hi.cuda()) & (wl.coarse.abs() >= 2.0 / M)
    d = torch.where(flip, -wl.coarse, wl.coarse)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = sg.correct_signs(d, wl.h)
    coarse_ms = 1e3 * (time.perf_counter() - t0)
    coarse_ok = bool(torch.equal(d, wl.coarse))
    del c, flip, d
    t = wl.grid.tables()
    inner = (t["pkg_type"].to(torch.int32) == 2)[:, None].expand(-1, 64)
    cells = t["pkg_cell"].view(torch.int32).to(torch.int64)
    cx, cy, cz = cells % M, (cells // M) % M, cells // (M * M)
    lo, hi = boxes(M)
    flip = inner & in_boxes(cx, cy, cz, lo.cuda(), hi.cuda())[:, None]
    phi = torch.where(flip, -wl.phi, wl.phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = sg.correct_package_signs(wl.grid, phi)
    pkg_ms = 1e3 * (time.perf_counter() - t0)
    pkg_ok = bool(torch.equal(phi, wl.phi))
    log(f"sign correction: coarse {coarse_ms:.2f} ms ({rc} rounds, repaired {coarse_ok}), "
        f"packages {pkg_ms:.2f} ms ({rp} rounds, repaired {pkg_ok})")
    return {"coarse_ms": coarse_ms, "coarse_rounds": rc, "coarse_repaired": coarse_ok,
            "packages_ms": pkg_ms, "package_rounds": rp, "packages_repaired": pkg_ok,
            "note": "signs flipped in 8 boxes away from the surface; wall time per call, outside the step; "
                    "'repaired' = the result equals the unbroken input, which the diffusion guarantees only for "
                    "a distance function (the displaced torus is not one)"}


def bench_single(args, log):
    import torch
    import paper_2512_11473_amd as sg
    import synth
    from paper_2512_11473_amd import workload

    cfg = synth.config_c5() if args.workload == "torus2048" else synth.config_c2()
    if args.n_iter is not None:
        cfg["n_iter"] = args.n_iter
    t0 = time.perf_counter()
    pos = synth.particles_for(cfg, args.particles)
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"], particles=pos)
    del pos
    setup_s = time.perf_counter() - t0
    log(f"{cfg['name']} set up in {setup_s:.1f}s: {wl.grid.n_packages} packages, {wl.grid.n_core} core")
    model, learned_info = (None, None) if args.no_learned else train_surrogate(args, log)
    # sweep configuration: tuned once on this grid (phi0 is only read), or fixed
    if args.sweep == "auto":
        tv, tg, ttab = sg.autotune_sweep(wl.grid, wl.phi0, wl.scratch, reps=10)
        tuned = {"variant": tv, "groups": tg, "source": "autotuned",
                 "us_per_sweep": {f"v{v}g{g}": float(x) for (v, g), x in zip(sg.SWEEP_TUNE_CANDIDATES, ttab)}}
    else:
        tv, tg = (int(x) for x in args.sweep.split(","))
        sg.set_sweep_config(tv, tg)
        tuned = {"variant": tv, "groups": tg, "source": "--sweep"}
    log(f"sweep configuration: variant {tv}, groups {tg}")
    P = wl.grid.n_packages
    n_core = wl.grid.n_core
    n_part = int(wl.pos.shape[0])
    integ = torch.empty((4, n_core * 64), device="cuda")
    packed = torch.empty((wl.grid.n_total, 64, 4), device="cuda")
    pos_sorted = torch.empty_like(wl.pos)
    perm = torch.empty(n_part, dtype=torch.int32, device="cuda")
    sort_ws = torch.empty(sg.sort_workspace_bytes(wl.grid, n_part), dtype=torch.uint8, device="cuda")
    n_fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    if args.overlap:   # the step on a stream of its own, the integrals on a second one
        torch.cuda.synchronize()
        torch.cuda.set_stream(torch.cuda.Stream())
    stream = torch.cuda.current_stream()

    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(2)] for k in
          ("build", "reinit", "grad", "sort", "probe", "integ")}
    acc = {k: 0.0 for k in ev}

    # with --overlap a second stream (default priority) takes the integrals,
    # which then run beside the gradient, the sort and the probe (memory-
    # bound); by default every step runs on one stream
    side = torch.cuda.Stream() if args.overlap else stream
    ev_reinit, ev_integ = torch.cuda.Event(), torch.cuda.Event()

    def step(record):
        def mark(k, i, st=stream):
            if record:
                ev[k][i].record(st)
        mark("build", 0)
        g = sg.build_packages(wl.coarse, wl.h)
        mark("build", 1)
        wl.phi.copy_(wl.phi0)
        mark("reinit", 0)
        sg.reinitialize(g, wl.phi, wl.scratch, cfg["n_iter"])
        mark("reinit", 1)
        ev_reinit.record(stream)
        side.wait_event(ev_reinit)
        mark("integ", 0, side)
        if model is not None:
            sg.compute_near_surface_integrals(g, wl.phi, integ, model=model, n_fallback=n_fb, stream=side)
        else:   # plain, factorised (its fractions go to the sweep's scratch)
            sg.compute_near_surface_integrals_factorised(g, wl.phi, wl.scratch, integ, stream=side)
        mark("integ", 1, side)
        ev_integ.record(side)
        mark("grad", 0)
        sg.compute_gradient_packed(g, wl.phi, packed)
        mark("grad", 1)
        mark("sort", 0)
        sg.sort_particles(g, wl.pos, pos_sorted, perm, workspace=sort_ws)
        mark("sort", 1)
        mark("probe", 0)
        sg.probe_particles_packed(g, packed, pos_sorted, wl.phi_p, wl.nrm_p)
        mark("probe", 1)
        stream.wait_event(ev_integ)
        return g

    for _ in range(args.warmup):
        step(False).destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = step(True)
        torch.cuda.synchronize()   # the build already synchronises once per step
        for k in ev:
            acc[k] += ev[k][0].elapsed_time(ev[k][1])
        g.destroy()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    fb_fraction = int(n_fb.item()) / max(1, n_core * 64) if model is not None else None

    # the same probe over the particles in generated order (not part of the step)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g = sg.build_packages(wl.coarse, wl.h)
    sg.reinitialize(g, wl.phi, wl.scratch, cfg["n_iter"])
    sg.compute_gradient_packed(g, wl.phi, packed)
    sg.probe_particles_packed(g, packed, wl.pos, wl.phi_p, wl.nrm_p)
    e0.record(stream)
    for _ in range(5):
        sg.probe_particles_packed(g, packed, wl.pos, wl.phi_p, wl.nrm_p)
    e1.record(stream)
    torch.cuda.synchronize()
    probe_random_ms = e0.elapsed_time(e1) / 5
    del pos_sorted, perm, sort_ws
    integrals = integrals_report(sg, g, wl, model, log)
    if learned_info is not None:
        integrals.update(learned_info)
    # grid-to-particle coupling of the integral field (Sec. 8), not part of the
    # step: the field at every activated point, then its probe at the particles
    field = torch.empty((g.n_total, 64, 4), device="cuda")
    fout = torch.empty((n_part, 4), device="cuda")
    sg.compute_integral_field(g, wl.phi, field)
    sg.probe_integral_field(g, field, wl.pos, fout)
    e2 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        sg.compute_integral_field(g, wl.phi, field)
    e1.record(stream)
    for _ in range(5):
        sg.probe_integral_field(g, field, wl.pos, fout)
    e2.record(stream)
    torch.cuda.synchronize()
    field_ms, fprobe_ms = e0.elapsed_time(e1) / 5, e1.elapsed_time(e2) / 5
    g.destroy()
    del field, fout
    multires = multires_build(sg, synth, cfg, wl.grid, log)
    signs = sign_correction(sg, cfg, wl, log)
    # a plain device copy of one field buffer into another (the sweep's streams
    # without its halos and face rows): the bandwidth this size reaches
    copy_reps = 20
    e0.record(stream)
    for _ in range(copy_reps):
        wl.scratch.copy_(wl.phi)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_us = e0.elapsed_time(e1) * 1e3 / copy_reps
    copy_gbps = 2 * wl.phi.numel() * wl.phi.element_size() / (copy_us * 1e-6) / 1e9

    K = args.steps
    ms_step = 1e3 * total_s / K
    upd_step = 64 * P * cfg["n_iter"]
    sort_ms, probe_ms = acc["sort"] / K, acc["probe"] / K
    probe_bytes = PROBE_BYTES_PER_PARTICLE * n_part + 16.0 * 64 * P
    reinit_ms = acc["reinit"] / K
    sweep_ms = reinit_ms / cfg["n_iter"]
    bytes_launch = REINIT_BYTES_PER_UPDATE * 64 * P
    achieved = bytes_launch / (sweep_ms * 1e-3) / 1e9
    rec = {
        "metric": "package-cell updates/s (reinit), probes/s; learned vs plain integral @1e-3",
        "value": upd_step / (ms_step * 1e-3),
        "unit": "package-cell updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[cfg["name"]],
                   "N": cfg["N"], "n_packages": P, "n_core": n_core, "n_iter": cfg["n_iter"],
                   "particles": n_part,
                   "integrals_in_step": "learned, gated, plain fallback" if model is not None
                   else "plain (factorised)"},
        "breakdown_ms": {k: acc[k] / K for k in acc},
        "reinit_updates_per_s": upd_step / (reinit_ms * 1e-3),
        "sweep_config": tuned,
        "probes_per_s": n_part / ((sort_ms + probe_ms) * 1e-3),
        "probe_particle_order": "sorted by home cell (Morton order) inside the step: sort + probe of the sorted particles",
        "probe_only_per_s": n_part / (probe_ms * 1e-3),
        "probes_per_s_generated_order": n_part / (probe_random_ms * 1e-3),
        "probe_hbm": {"algorithmic_bytes_per_launch": probe_bytes,
                      "note": "28 B per particle (position in, value and normal out) plus the packed field once",
                      "sorted_probe_GBps": probe_bytes / (probe_ms * 1e-3) / 1e9,
                      "sorted_probe_frac": probe_bytes / (probe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "sort_plus_probe_GBps": probe_bytes / ((sort_ms + probe_ms) * 1e-3) / 1e9,
                      "generated_order_GBps": probe_bytes / (probe_random_ms * 1e-3) / 1e9},
        "integral_cells_per_s_in_step": n_core * 64 / (acc["integ"] / K * 1e-3),
        "step_fallback_fraction": fb_fraction,
        "integrals": integrals,
        "multires_build": multires,
        "sign_correction": signs,
        "integral_field": {"field_ms": field_ms, "field_points_per_s": 64 * P / (field_ms * 1e-3),
                           "probe_ms": fprobe_ms, "probes_per_s": n_part / (fprobe_ms * 1e-3),
                           "note": "(K_W, h K_grad) at every activated point, then interpolated to the particles "
                                   "(generated order); measured outside the step"},
        "roofline": {"bound": "hbm", "kernel": f"reinit sweep (variant {tv}, groups {tg})", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"reinit_sweep_{cfg['name']}_counters.txt", f"v{tv}g{tg}"),
                     "avg_launch_us": sweep_ms * 1e3, "algorithmic_bytes_per_launch": bytes_launch,
                     "copy_same_size_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                     "note": ("phi ping-pong of 64 MB is resident in the 256 MB Infinity Cache"
                              if cfg["name"] == "prism512" else
                              "phi ping-pong of 0.9 GB streams from HBM")},
        "setup_s": setup_s,
    }
    log(f"timed {K} steps: {ms_step:.2f} ms per step")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(cfg, args.cpu_iters or cfg["n_iter"], args.cpu_seconds)
        log("cpu baseline done")
    return rec


def bench_batch(args, log):
    import numpy as np
    import torch
    import synth
    from paper_2512_11473_amd import workload

    cfg = synth.config_c3()
    n_iter = args.n_iter or cfg["n_iter"]
    t0 = time.perf_counter()
    bw = workload.setup_batch(cfg["shapes"], cfg["noise_amp"])
    setup_s = time.perf_counter() - t0
    v, b, table = bw.batch.autotune(bw.phi0, bw.scratch, reps=5)
    counts = [p.grid.n_packages for p in bw.parts]
    for _ in range(args.warmup):
        bw.reset()
        bw.batch.reinitialize(bw.phi, bw.scratch, n_iter, use_graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bw.phi.copy_(bw.phi0)
        e0.record()
        bw.batch.reinitialize(bw.phi, bw.scratch, n_iter, use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
    total_s = time.perf_counter() - t0
    K = args.steps
    upd = 64 * bw.batch.n_work * n_iter
    sweep_ms = ms / K / n_iter
    achieved = REINIT_BYTES_PER_UPDATE * 64 * bw.batch.n_work / (sweep_ms * 1e-3) / 1e9
    return {
        "metric": "package-cell updates/s (reinit), probes/s; learned vs plain integral @1e-3",
        "value": upd / (ms / K * 1e-3), "unit": "package-cell updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": 1e3 * total_s / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64: 64 seeded random unions at 64^3..512^3, one persistent launch per "
                               "iteration over a global worklist, 50 iterations replayed as a HIP graph",
                   "n_shapes": len(counts), "n_packages": int(bw.batch.n_work), "n_iter": n_iter,
                   "packages_min": int(min(counts)), "packages_max": int(max(counts))},
        "autotuned": {"variant": ["dpp", "lds"][v], "blocks_per_cu": b if b else "one wavefront per 4 packages",
                      "us_per_sweep": {f"{['dpp', 'lds'][i]}_{'bpc%d' % bb if bb else 'flat'}": float(table[i, j])
                                       for i in range(2) for j, bb in enumerate((1, 2, 4, 8, 16, 0))}},
        "roofline": {"bound": "hbm", "kernel": "batched sweep", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": sweep_ms * 1e3},
        "setup_s": setup_s,
    }


# Tab. 1 of the paper: CPU timings of its timing test (unit not stated), context only
PAPER_TAB1 = {"sequential_1_thread": 22.948, "sequential_4_threads": 7.429,
              "stencil_1_thread": 59.972, "stencil_4_threads": 21.378,
              "note": "SPHinXsys on an unnamed CPU; the paper gives no unit and no repetition count"}
SHELL_CROPS = [(175, 96, 96), (96, 175, 96), (96, 96, 175), (17, 96, 96)]


def bench_shell(args, log):
    """The paper's timing test (Sec. 9, Tab. 1) on the shell at 1/1024: the
    sequential update and the seven-point Laplacian over all activated data."""
    import torch
    import paper_2512_11473_amd as sg
    import synth
    from paper_2512_11473_amd import workload

    cfg = synth.config_shell()
    t0 = time.perf_counter()
    wl = workload.setup(cfg["shape"], cfg["N"], cfg["noise_amp"], cfg["noise_seed"])
    setup_s = time.perf_counter() - t0
    g = wl.grid
    P = g.n_packages
    out = torch.empty_like(wl.phi)
    stream = torch.cuda.current_stream()
    # the sweep configuration also fixes the package order of the stencil pass
    if args.sweep == "auto":
        tv, tg, _ = sg.autotune_sweep(g, wl.phi, wl.scratch, reps=10)
        source = "autotuned"
    else:
        tv, tg = (int(x) for x in args.sweep.split(","))
        sg.set_sweep_config(tv, tg)
        source = "--sweep"
    for _ in range(args.warmup):
        sg.sequential_update(g, wl.phi, cfg["delta"])
        sg.compute_laplacian(g, wl.phi, out)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        sg.sequential_update(g, wl.phi, cfg["delta"])
        ev[k][1].record(stream)
        sg.compute_laplacian(g, wl.phi, out)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    K = args.steps
    seq_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / K
    lap_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / K
    pts = 64 * P
    lap_bytes = REINIT_BYTES_PER_UPDATE * pts
    seq_bytes = 8.0 * pts
    rec = {
        "metric": "active points/s of the seven-point Laplacian (paper's timing test)",
        "value": pts / (lap_ms * 1e-3), "unit": "points/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": 1e3 * total_s / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "shell1024: spherical shell of radii 0.3 and 0.31 about (0.5, 0.5, 0.5) at 1/1024, "
                               "phi = its signed distance; one step = sequential update (phi += 1e-6) and "
                               "seven-point Laplacian over all activated data",
                   "N": cfg["N"], "n_packages": P, "points": pts},
        "sequential_ms": seq_ms, "laplacian_ms": lap_ms,
        "sweep_config": {"variant": tv, "groups": tg, "source": source},
        "sequential_points_per_s": pts / (seq_ms * 1e-3),
        "roofline": {"bound": "hbm", "kernel": "laplacian", "achieved": lap_bytes / (lap_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": lap_bytes / (lap_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic("laplacian_shell1024_counters.txt",
                                                 "worklist" if tv in (3, 4) else "linear"),
                     "algorithmic_bytes_per_launch": lap_bytes},
        "sequential_roofline": {"achieved": seq_bytes / (seq_ms * 1e-3) / 1e9, "unit": "GB/s",
                                "frac": seq_bytes / (seq_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "algorithmic_bytes_per_launch": seq_bytes},
        "paper_tab1_cpu": PAPER_TAB1,
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        import oracle
        runs = [oracle.setup_crop(cfg["shape"], cfg["N"], o, 64, cfg["noise_amp"], cfg["noise_seed"])
                for o in SHELL_CROPS]
        dense = [oracle.dense_state(r.tab, r.active, r.phi0, r.B) for r in runs]
        oracle.laplacian(runs[0].N, runs[0].h, runs[0].B, runs[0].active, dense[0])
        done, secs, passes = 0, 0.0, 0
        while secs < args.cpu_seconds:
            r, d = runs[passes % len(runs)], dense[passes % len(runs)]
            t1 = time.perf_counter()
            oracle.laplacian(r.N, r.h, r.B, r.active, d)
            secs += time.perf_counter() - t1
            done += len(r.active)
            passes += 1
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        rec["cpu_baseline"] = {"value": done / secs, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": f"{passes} FP64 Laplacian passes of the oracle over 64^3-coarse-cell crops "
                                         f"of the shell band in turn ({secs:.1f} s)"}
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path has no multi-GPU mode",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batch64":
        rec = bench_batch(args, log)
    elif args.workload == "shell1024":
        rec = bench_shell(args, log)
    else:
        rec = bench_single(args, log)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
