#!/usr/bin/env python3
"""Benchmark: FP64 cell-updates/s of the SSP2(222) IMEX step on one MI355X.

Workload: 2-D resistive single-fluid Kelvin-Helmholtz set-up, 256 x 512 cells on
[-1/2, 1/2] x [-1, 1], periodic, Gamma = 4/3, sigma = 1e3, seeded random v_y perturbation,
FP64 (the configuration the headline metric is quoted on).  One step = one full
SSP2(222) IMEX step over the whole grid: two implicit-stage solves (Newton per cell with
nested primitive recovery), two FVS + WENO3 flux passes fused with the stage combiners,
and the primitive recovery of the new state.  State is resident in HBM throughout.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def cpu_baseline(budget_s: float = 12.0, single_core_budget_s: float = 8.0) -> dict:
    """The CPU oracle on the same workload: on all of this host's cores (OpenMP over cells),
    then on one core (the paper's serial reference point)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle import oracle as O
    from oracle_runs import advance, initial_state
    from paper_1808_09721_amd import workloads as WL
    wl = WL.kelvin_helmholtz_2d()

    def run(budget):
        g, cons, prims = initial_state(wl)
        dt = O.dt(g, wl.cfl)
        t0 = time.perf_counter()
        advance(g, cons, prims, dt, steps=1)
        t1 = time.perf_counter() - t0
        steps = max(1, min(100, int(budget / max(t1, 1e-3))))
        t0 = time.perf_counter()
        advance(g, cons, prims, dt, steps=steps)
        return steps, time.perf_counter() - t0

    cores = O.set_threads(0)
    steps, el = run(budget_s)
    O.set_threads(1)
    steps1, el1 = run(single_core_budget_s)
    O.set_threads(cores)
    return {"value": wl.cells * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"kelvin_helmholtz_2d 256x512, {steps} SSP2(222) steps after 1 untimed, "
                      f"OpenMP over cells ({cores} threads), {el:.1f} s",
            "single_core": {"value": wl.cells * steps1 / el1, "unit": "cell-updates/s", "cores": 1,
                            "sample": f"kelvin_helmholtz_2d 256x512, {steps1} steps after 1 untimed, {el1:.1f} s"}}


# sources of the single-grid kernels (the headline workload's kernels)
SINGLE_GRID_SOURCES = ("physics.hpp", "stage.hpp", "kernels.hpp", "rmhd.hip")


def source_hash() -> str:
    """Hash of the single-grid HIP sources; counter-derived traffic is reported only while it
    matches the hash recorded with the counters."""
    import hashlib
    h = hashlib.sha256()
    for f in SINGLE_GRID_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1808_09721_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(tag: str, kernel_prefix: str):
    """HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE) recorded under profiles/,
    averaged over the kernels whose names start with kernel_prefix (both flux passes of a
    step, as the per-launch time is their average)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    vals = [v["fetch_bytes"] + v["write_bytes"] for k, v in rec["kernels"].items() if k.startswith(kernel_prefix)]
    return sum(vals) / len(vals) if vals else None


def batched_measure(steps: int, warmup: int) -> dict:
    """The 64-domain batched workload (32 1-D shock tubes, N ~ U[128, 4096]; 32 2-D KH set-ups,
    sides ~ U[64, 512]; sigma ~ 10^U[1, 6]; seed 4): one batched step (autotuned, graph-
    captured) against the same domains stepped one after another on the single-grid path."""
    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    doms = WL.batched_domains(seed=4)
    cells = sum(w.cells for w in doms)
    B = R.Batch(doms)
    tuning = B.autotune()
    for _ in range(warmup):
        B.step()
    B.stats(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        B.step()
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    st = B.stats(reset=True)
    B.set_stats_detail(True)          # one untimed step for the step-count histogram
    B.step()
    sd = B.stats(reset=True)
    B.close()
    # the same domains, one single-grid context each, stepped in turn
    solvers = []
    for wl in doms:
        s = R.Solver(R.params_from(wl))
        c, w = s.initial_state(wl.prims, wl.EB)
        solvers.append((s, c, w, s.dt()))
    for _ in range(warmup):
        for s, c, w, h in solvers:
            s.step(h, c, w)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        for s, c, w, h in solvers:
            s.step(h, c, w)
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / steps
    for s, *_ in solvers:
        s.close()
    return {"workload": "64 domains (32 x 1-D Brio-Wu N~U[128,4096], 32 x 2-D KHI sides~U[64,512], "
                        "sigma~10^U[1,6], seed 4)", "cells": cells,
            "value": cells / (ms_b / 1e3), "unit": "cell-updates/s", "ms_per_step": ms_b,
            "plain_value": cells / (ms_p / 1e3), "plain_ms_per_step": ms_p, "speedup_vs_plain": ms_p / ms_b,
            "newton_iters_per_cell_stage": st["newton_iters"] / max(1, st["stage_cells"]),
            "newton_iters_p50": R.newton_percentile(sd, 0.5), "newton_iters_p99": R.newton_percentile(sd, 0.99),
            "final_residual_max": sd["residual_max"],
            "newton_iters_max": st["newton_max"], "failures": st["failures"], "tuning": tuning}


def learned_measure(steps: int, warmup: int, n: int = 1024, train_n: int = 512, train_seeds=(1, 2, 3, 4),
                    harvest_steps: int = 6, dt_factors=(1.0, 0.5, 0.25), epochs: int = 8) -> dict:
    """Learned starting guess on the two-fluid current sheet with sigma ~ 10^U[2, 6] per cell:
    harvest (features, target) rows from train_n^2 runs at seeds 1-4 whose steps cycle through
    dt_factors times the CFL step (so the network sees the stage coefficient of finer grids),
    fit the normalisation, train on the device, then time ``steps`` steps of the n^2 set-up at
    the held-out seed 5 with the plain and with the learned guess (same initial state, same
    dt).  Harvest and training are outside the timed regions and reported separately."""
    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    t0 = time.perf_counter()
    X, T = R.harvest_stages([WL.learned_guess_sheet(train_n, seed=sd, steps=harvest_steps) for sd in train_seeds],
                            harvest_steps, dt_factors)
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    off = X.shape[0]
    net = R.Mlp(WL.mlp_initial_params(7))
    net.fit_norm(X, T)
    t1 = time.perf_counter()
    hist = net.train(X, T, batch=16384, epochs=epochs, lr0=3e-3, lr1=1e-4, seed=11)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del X, T

    wl = WL.learned_guess_sheet(n, seed=5, steps=steps)
    res = {}
    for mode in ("plain_queue", "plain", "learned"):
        s = R.Solver.for_workload(wl)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        if mode == "plain_queue":
            s.set_newton_cap(1)        # the stage queue after one Newton step (plain default: none)
        if mode == "learned":
            s.set_guess_model(net)
        for _ in range(warmup):
            s.step(dt, c, w)
        s.stats(reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            s.step(dt, c, w)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = s.stats(reset=True)
        R.rmhd_set_timing(s.ctx, True)
        R.rmhd_get_timing(s.ctx, reset=True)
        for _ in range(2):
            s.step(dt, c, w)
        tm = R.rmhd_get_timing(s.ctx, reset=True)
        R.rmhd_set_timing(s.ctx, False)
        s.stats(reset=True)
        s.set_stats_detail(True)
        s.step(dt, c, w)
        sd = s.stats(reset=True)
        res[mode] = {"ms_per_step": ms, "value": wl.cells / (ms / 1e3),
                     "newton_iters_per_cell_stage": st["newton_iters"] / max(1, st["stage_cells"]),
                     "newton_iters_p50": R.newton_percentile(sd, 0.5),
                     "newton_iters_p99": R.newton_percentile(sd, 0.99),
                     "residual_evals_per_cell_stage": st["residual_evals"] / max(1, st["stage_cells"]),
                     "final_residual_max": sd["residual_max"],
                     "c2p_iters_per_cell_stage": st["c2p_iters"] / max(1, st["stage_cells"]),
                     "newton_iters_max": st["newton_max"], "failures": st["failures"],
                     "stage_ms_per_launch": tm["stage_ms"] / tm["stage_launches"]}
        s.close()
    net.close()
    return {"workload": f"two-fluid current sheet {n}x{n}, sigma~10^U[2,6] per cell, seed 5 (held out)",
            "cells": wl.cells, "unit": "cell-updates/s", "steps": steps,
            "value": res["learned"]["value"], "plain_value": res["plain"]["value"],
            "speedup_vs_plain": res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"],
            "plain": res["plain"], "learned": res["learned"], "plain_queue": res["plain_queue"],
            "training": {"rows": off, "harvest": f"{len(train_seeds)} seeds x {harvest_steps} steps x 2 stages of "
                                                 f"{train_n}x{train_n}, dt factors {list(dt_factors)}",
                         "epochs": epochs, "batch": 16384,
                         "loss_first_epoch": float(hist[0]), "loss_last_epoch": float(hist[-1]),
                         "harvest_s": t_harvest, "train_s": t_train}}


def ssp3_measure(steps: int, warmup: int) -> dict:
    """SSP3(332) (three implicit stages and three flux passes per step) on the headline KHI
    grid and on the two-fluid sheet at 1024^2 with sigma ~ 10^U[2, 6] per cell."""
    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    out = {}
    for name, wl in (("kelvin_helmholtz_2d 256x512", WL.kelvin_helmholtz_2d()),
                     ("two-fluid current sheet 1024x1024, sigma~10^U[2,6] per cell", WL.learned_guess_sheet(1024))):
        s = R.Solver.for_workload(wl, integrator=R.SSP3_332)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        n = steps if wl.cells < 500000 else max(3, steps // 10)
        for _ in range(warmup):
            s.step(dt, c, w)
        s.stats(reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            s.step(dt, c, w)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        st = s.stats(reset=True)
        out[name] = {"cells": wl.cells, "steps": n, "ms_per_step": ms, "value": wl.cells / (ms / 1e3),
                     "unit": "cell-updates/s", "newton_iters_per_cell_stage": st["newton_iters"] / max(1, st["stage_cells"]),
                     "failures": st["failures"]}
        s.close()
    return out


def grid3d_measure(steps: int, warmup: int) -> dict:
    """3-D grids (SSP2(222)): Kelvin-Helmholtz 128 x 256 x 128 (single fluid, 4.2 M cells) and
    the two-fluid sheet at 128^3 (2.1 M cells); and one y-slab of the two-fluid 1024^2 sheet
    as eight GPUs would hold it (1024 x 128 cells, sigma ~ 10^U[2, 6] per cell), the shape a
    sharded step runs on each GPU.  Per-kernel times from a separate timed pass."""
    import numpy as np
    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    slab = WL.learned_guess_sheet(1024)
    slab = WL.Workload("two-fluid sheet slab", slab.model, 2, 1024, 128, slab.x0, slab.x1, slab.y0,
                       slab.y0 + (slab.y1 - slab.y0) / 8, gamma=slab.gamma, sigma=slab.sigma, bc=slab.bc,
                       mu1=slab.mu1, mu2=slab.mu2, prims=np.ascontiguousarray(slab.prims[:, :128]),
                       EB=np.ascontiguousarray(slab.EB[:, :128]),
                       sigma_cell=np.ascontiguousarray(slab.sigma_cell[:128]))
    out = {}
    for name, wl in (("kelvin_helmholtz_3d 128x256x128", WL.kelvin_helmholtz_3d()),
                     ("two_fluid_sheet_3d 128x128x128", WL.two_fluid_sheet_3d(128, 128, 128)),
                     ("two-fluid sheet 1024x128 (one of 8 y-slabs of 1024^2, sigma~10^U[2,6])", slab)):
        s = R.Solver.for_workload(wl)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        n = max(3, steps)
        for _ in range(warmup):
            s.step(dt, c, w)
        s.stats(reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            s.step(dt, c, w)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        st = s.stats(reset=True)
        R.rmhd_set_timing(s.ctx, True)
        R.rmhd_get_timing(s.ctx, reset=True)
        for _ in range(3):
            s.step(dt, c, w)
        tm = R.rmhd_get_timing(s.ctx, reset=True)
        R.rmhd_set_timing(s.ctx, False)
        out[name] = {"cells": wl.cells, "steps": n, "ms_per_step": ms, "value": wl.cells / (ms / 1e3),
                     "unit": "cell-updates/s",
                     "newton_iters_per_cell_stage": st["newton_iters"] / max(1, st["stage_cells"]),
                     "failures": st["failures"],
                     "stage_ms_per_launch": tm["stage_ms"] / max(1, tm["stage_launches"]),
                     "flux_ms_per_pass": tm["flux_ms"] / max(1, tm["flux_launches"]),
                     "c2p_ms_per_launch": tm["c2p_ms"] / tm["c2p_launches"] if tm["c2p_launches"] else None}
        s.close()
    return out


def ideal_measure(steps: int, warmup: int, resistive_ms: float) -> dict:
    """The ideal model (explicit steps) on the headline Kelvin-Helmholtz grid with both
    tableaux, and on the 3-D grid, against the resistive single-fluid IMEX step on the same
    2-D grid (the paper reports resistive IMEX runs often taking over ten times longer than
    ideal explicit ones)."""
    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    out = {}
    for name, wl, integ in (("kelvin_helmholtz_2d 256x512 ideal, SSP2 explicit", WL.kelvin_helmholtz_2d(), R.SSP2_222),
                            ("kelvin_helmholtz_2d 256x512 ideal, SSP3 explicit", WL.kelvin_helmholtz_2d(), R.SSP3_332),
                            ("kelvin_helmholtz_3d 128x256x128 ideal, SSP2 explicit", WL.kelvin_helmholtz_3d(),
                             R.SSP2_222)):
        wl = WL.as_ideal(wl)
        s = R.Solver.for_workload(wl, integrator=integ)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        n = steps if wl.cells < 500000 else max(3, steps // 20)
        for _ in range(warmup):
            s.step(dt, c, w)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            s.step(dt, c, w)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        R.rmhd_set_timing(s.ctx, True)
        R.rmhd_get_timing(s.ctx, reset=True)
        for _ in range(3):
            s.step(dt, c, w)
        tm = R.rmhd_get_timing(s.ctx, reset=True)
        R.rmhd_set_timing(s.ctx, False)
        out[name] = {"cells": wl.cells, "steps": n, "ms_per_step": ms, "value": wl.cells / (ms / 1e3),
                     "unit": "cell-updates/s", "flux_ms_per_pass": tm["flux_ms"] / max(1, tm["flux_launches"]),
                     "c2p_ms_per_launch": tm["c2p_ms"] / tm["c2p_launches"] if tm["c2p_launches"] else None}
        s.close()
    out["resistive_over_ideal_step_time_2d_ssp2"] = resistive_ms / out[
        "kelvin_helmholtz_2d 256x512 ideal, SSP2 explicit"]["ms_per_step"]
    return out


def filled_measure(warmup: int) -> dict:
    """Kernel efficiency when the grid fills the GPU (the 256 x 512 headline grid gives each
    SIMD about two wavefronts): the two-fluid sheet at 1024^2 (sigma ~ 10^U[2, 6] per cell;
    working set of a flux pass ~0.6 GB, above the 256 MB last-level cache) and the
    single-fluid Kelvin-Helmholtz set-up at 128 x 256 x 128.  Stage: algorithmic FP64 FLOPs
    (perfmodel, from the measured iteration counts) per second against the FP64 vector peak;
    flux pass: algorithmic bytes of a fused pass per second against HBM peak."""
    from paper_1808_09721_amd import perfmodel as PM
    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    out = {}
    for name, wl in (("two-fluid sheet 1024x1024, sigma~10^U[2,6]", WL.learned_guess_sheet(1024)),
                     ("kelvin_helmholtz_3d 128x256x128", WL.kelvin_helmholtz_3d())):
        s = R.Solver.for_workload(wl)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        for _ in range(warmup):
            s.step(dt, c, w)
        s.stats(reset=True)
        R.rmhd_set_timing(s.ctx, True)
        R.rmhd_get_timing(s.ctx, reset=True)
        for _ in range(5):
            s.step(dt, c, w)
        tm = R.rmhd_get_timing(s.ctx, reset=True)
        R.rmhd_set_timing(s.ctx, False)
        st = s.stats(reset=True)
        stage_ms = tm["stage_ms"] / tm["stage_launches"]
        flux_ms = tm["flux_ms"] / tm["flux_launches"]
        flops = PM.stage_flops(wl.model, st["stage_cells"], st["residual_evals"], st["newton_iters"], st["c2p_iters"])
        tf = flops / tm["stage_launches"] / (stage_ms / 1e3) / 1e12
        fb = 0.5 * (PM.flux_bytes_per_cell(wl.model, "first") + PM.flux_bytes_per_cell(wl.model, "second"))
        if wl.ndim == 3:   # primitives recovered by the recovery kernel, not the flux pass
            fb -= 0.5 * 8 * PM.NPRIM[wl.model]
        gbs = fb * wl.cells / (flux_ms / 1e3) / 1e9
        out[name] = {"cells": wl.cells,
                     "implicit_stage": {"ms_per_launch": stage_ms, "achieved": tf, "unit": "TFLOP/s",
                                        "peak": PM.PEAK_FP64_VECTOR_TFLOPS, "frac": tf / PM.PEAK_FP64_VECTOR_TFLOPS,
                                        "flops_per_cell": flops / st["stage_cells"]},
                     "flux": {"ms_per_pass": flux_ms, "achieved": gbs, "unit": "GB/s", "peak": PM.PEAK_HBM_GBS,
                              "frac": gbs / PM.PEAK_HBM_GBS, "bytes_per_cell": fb}}
        s.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-ssp3", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-ideal", action="store_true")
    ap.add_argument("--no-filled", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (traffic calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(the path shards by domain slabs, see DESIGN.md)", file=sys.stderr)
        return 2

    import torch

    from paper_1808_09721_amd import perfmodel as PM
    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL

    torch.cuda.set_device(0)
    wl = WL.kelvin_helmholtz_2d()
    solver = R.Solver(R.params_from(wl))
    cons, prims = solver.initial_state(wl.prims, wl.EB)
    dt = solver.dt()
    for _ in range(args.warmup):
        solver.step(dt, cons, prims)
    solver.stats(reset=True)

    # timed region: K whole steps on torch's current stream (the library's stream)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        solver.step(dt, cons, prims)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1)
    st = solver.stats(reset=True)
    cells = wl.cells
    value = cells * args.steps / (ms / 1e3)
    # four more timed regions of the same length, for the median of five
    runs = [ms / args.steps]
    for _ in range(4):
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            solver.step(dt, cons, prims)
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1) / args.steps)
    solver.stats(reset=True)

    # per-kernel pass: HIP events around every launch on the same stream
    if args.copy_mib:
        src = torch.empty(args.copy_mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    args.timing_steps = max(1, args.timing_steps)
    R.rmhd_set_timing(solver.ctx, True)
    R.rmhd_get_timing(solver.ctx, reset=True)
    for _ in range(args.timing_steps):
        solver.step(dt, cons, prims)
    tm = R.rmhd_get_timing(solver.ctx, reset=True)
    st2 = solver.stats(reset=True)
    R.rmhd_set_timing(solver.ctx, False)
    # step-count histogram and residual maximum from two more steps, outside every timing
    solver.set_stats_detail(True)
    for _ in range(2):
        solver.step(dt, cons, prims)
    st3 = solver.stats(reset=True)
    solver.set_stats_detail(False)
    stage_ms = tm["stage_ms"] / tm["stage_launches"]
    flux_ms = tm["flux_ms"] / tm["flux_launches"]
    c2p_ms = tm["c2p_ms"] / tm["c2p_launches"] if tm["c2p_launches"] else None
    flops = PM.stage_flops(wl.model, st2["stage_cells"], st2["residual_evals"], st2["newton_iters"],
                           st2["c2p_iters"])
    stage_tflops = flops / tm["stage_launches"] / (stage_ms / 1e3) / 1e12
    flux_bytes = 0.5 * (PM.flux_bytes_per_cell(wl.model, "first") + PM.flux_bytes_per_cell(wl.model, "second"))
    flux_gbs = flux_bytes * cells / (flux_ms / 1e3) / 1e9
    kernels = {
        "implicit_stage": {"bound": "alu", "achieved": stage_tflops, "peak": PM.PEAK_FP64_VECTOR_TFLOPS,
                           "unit": "TFLOP/s", "frac": stage_tflops / PM.PEAK_FP64_VECTOR_TFLOPS,
                           "ms_per_launch": stage_ms, "flops_per_cell": flops / st2["stage_cells"]},
        "flux": {"bound": "hbm", "achieved": flux_gbs, "peak": PM.PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": flux_gbs / PM.PEAK_HBM_GBS, "ms_per_launch": flux_ms, "bytes_per_cell": flux_bytes},
        "c2p": {"ms_per_launch": c2p_ms,
                "note": "recovered inside the second flux pass" if c2p_ms is None else "separate kernel"},
    }
    dominant = "implicit_stage" if 2 * stage_ms >= 2 * flux_ms else "flux"
    roof = {k: kernels[dominant][k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof["kernel"] = dominant
    roof["traffic"] = measured_traffic("khi_256x512", "rmhd::k_flux<0, 2, 64, 16" if dominant == "flux" else "rmhd::k_stage<0>")
    if roof["traffic"] is not None and dominant == "flux":
        roof["traffic_over_algorithmic"] = roof["traffic"] / (flux_bytes * cells)

    out = {
        "metric": "FP64 cell-updates/s per IMEX step + Newton iters/cell, plain vs batched+learned",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "kelvin_helmholtz_2d 256x512 resistive single fluid, sigma=1e3, periodic, "
                               "SSP2(222) IMEX + FVS/WENO3, plain form", "cells": cells,
                   "parallelism": "single GPU"},
        "ms_per_step_runs": runs,
        "value_median_of_5": cells / (sorted(runs)[2] / 1e3),
        "newton_iters_per_cell_stage": st["newton_iters"] / max(1, st["stage_cells"]),
        "newton_iters_p50": R.newton_percentile(st3, 0.5),
        "newton_iters_p99": R.newton_percentile(st3, 0.99),
        "newton_iters_max": st["newton_max"],
        "final_residual_max": st3["residual_max"],
        "c2p_iters_per_residual": st["c2p_iters"] / max(1, st["residual_evals"]),
        "failures": st["failures"],
        "wall_s": wall,
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_batched:
        out["batched"] = batched_measure(max(5, args.steps // 5), args.warmup)
    if not args.no_learned:
        out["learned"] = learned_measure(10, args.warmup)
    if not args.no_ssp3:
        out["ssp3"] = ssp3_measure(max(10, args.steps // 2), args.warmup)
    if not args.no_3d:
        out["grid3d"] = grid3d_measure(max(3, args.steps // 20), args.warmup)
    if not args.no_ideal:
        out["ideal"] = ideal_measure(max(10, args.steps // 2), args.warmup, ms / args.steps)
    if not args.no_filled:
        out["filled"] = filled_measure(args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["gpu_speedup"] = value / out["cpu_baseline"]["value"]
        out["cpu_baseline"]["single_core"]["gpu_speedup"] = value / out["cpu_baseline"]["single_core"]["value"]
    print(json.dumps(out), flush=True)
    solver.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
