#!/usr/bin/env python3
"""Benchmark: FP64 cell-updates/s of the SSP2(222) IMEX step on one MI355X, plain form and
learned form.

Headline workload: two-fluid resistive RMHD current sheet, 1024 x 1024 periodic cells on
[-1/2, 1/2)^2, charge-to-mass ratios +-1000, Gamma = 4/3, rho_s = p_s = 1, conductivity
10^U[2, 6] per cell (eta = 1/sigma), seeded velocity noise (seed 5, held out of the
network's training rows), FP64.  One step = one full SSP2(222) IMEX step over the whole
grid: two implicit-stage solves (Newton per cell with the nested primitive recovery), two
FVS + WENO3 flux passes fused with the stage combiners, and the primitive recovery of the
new state.  `value` is the plain form (Newton from the stage's right-hand side, the library
default); the learned form (the network's starting guess, the same FP64 Newton to the same
1e-12 residual) is on the same line.  State is resident in HBM throughout; the network is
trained on the device before its timed region.  The other configurations (1-D Brio-Wu tube, 2-D Kelvin-Helmholtz
256 x 512, two-fluid sheet 512^2, the 64-domain batch) are reported as secondary fields.

Prints one JSON line.  ``--gpus`` above 1 is refused: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def cpu_baseline(budget_s: float = 10.0) -> dict:
    """The CPU oracle on the headline workload (two-fluid sheet 1024^2, per-cell sigma, seed
    5): SSP2(222) steps of the whole grid on all of this host's cores (OpenMP over cells), then
    one step on one core (the paper's serial reference point) of a 1024 x 128 slab of the same
    initial data."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np

    from oracle import oracle as O
    from oracle_runs import advance, initial_state
    from paper_1808_09721_amd import workloads as WL
    wl = WL.learned_guess_sheet(1024, seed=5, steps=1)
    cores = O.set_threads(0)
    g, cons, prims = initial_state(wl)
    dt = O.dt(g, wl.cfl)
    t0 = time.perf_counter()
    advance(g, cons, prims, dt, steps=1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(5, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    advance(g, cons, prims, dt, steps=steps)
    el = time.perf_counter() - t0
    slab = WL.Workload("two-fluid sheet slab", wl.model, 2, 1024, 128, wl.x0, wl.x1, wl.y0,
                       wl.y0 + (wl.y1 - wl.y0) / 8, gamma=wl.gamma, sigma=wl.sigma, bc=wl.bc, mu1=wl.mu1,
                       mu2=wl.mu2, prims=np.ascontiguousarray(wl.prims[:, :128]),
                       EB=np.ascontiguousarray(wl.EB[:, :128]), sigma_cell=np.ascontiguousarray(wl.sigma_cell[:128]))
    O.set_threads(1)
    g1, c1, p1 = initial_state(slab)
    t0 = time.perf_counter()
    advance(g1, c1, p1, dt, steps=1)
    el1 = time.perf_counter() - t0
    O.set_threads(cores)
    return {"value": wl.cells * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"two-fluid sheet 1024x1024 per-cell sigma, {steps} SSP2(222) steps after 1 untimed, "
                      f"OpenMP over cells ({cores} threads), {el:.1f} s",
            "single_core": {"value": slab.cells / el1, "unit": "cell-updates/s", "cores": 1,
                            "sample": f"1 SSP2(222) step of a 1024x128 slab (first 128 rows) of the same "
                                      f"initial data, same dt, {el1:.1f} s"}}


# sources of the single-grid kernels (the headline workload's kernels)
SINGLE_GRID_SOURCES = ("physics.hpp", "stage.hpp", "lu.hpp", "kernels.hpp", "rmhd.hip", "mlp.hip", "mlp_net.hpp")


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


def copy_calibration(mib: int) -> None:
    """A fill and a plain device copy of ``mib`` MiB: kernels of known traffic against which
    the HBM counters of a profiled run are scaled (nothing when mib is 0)."""
    if not mib:
        return
    import torch
    src = torch.empty(mib << 17, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def timed_steps(step, steps: int) -> float:
    """Milliseconds per step of ``steps`` calls of step(), between HIP events on torch's
    current stream (the library's), synchronised on both sides."""
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def newton_fields(R, st: dict, sd: dict) -> dict:
    """Newton statistics of a counted run (st) and of a detailed one (sd: histogram, residual)."""
    n = max(1, st["stage_cells"])
    return {"newton_iters_per_cell_stage": st["newton_iters"] / n,
            "jacobians_per_cell_stage": st["jacobian_evals"] / n,
            "residual_evals_per_cell_stage": st["residual_evals"] / n,
            "c2p_iters_per_cell_stage": st["c2p_iters"] / n,
            "newton_iters_p50": R.newton_percentile(sd, 0.5), "newton_iters_p99": R.newton_percentile(sd, 0.99),
            "newton_iters_max": st["newton_max"], "final_residual_max": sd["residual_max"],
            "failures": st["failures"]}


def measure_form(wl, steps: int, warmup: int, runs: int = 5, timing_steps: int = 10, net=None, cap=None,
                 integrator=0) -> dict:
    """One workload on the single-grid path: ``runs`` timed regions of ``steps`` steps after
    ``warmup`` steps (the first region is the reported one), then a pass with HIP events
    around every launch (per-kernel times and the counters of the same launches), then two
    steps with the detailed statistics."""
    from paper_1808_09721_amd import perfmodel as PM
    from paper_1808_09721_amd import rmhd as R
    s = R.Solver.for_workload(wl, integrator=integrator)
    c, w = s.initial_state(wl.prims, wl.EB)
    dt = s.dt()
    if net is not None:
        s.set_guess_model(net)
    if cap is not None:
        s.set_newton_cap(cap)
    for _ in range(warmup):
        s.step(dt, c, w)
    s.stats(reset=True)
    ms = [timed_steps(lambda: s.step(dt, c, w), steps)]
    st = s.stats(reset=True)
    for _ in range(runs - 1):
        ms.append(timed_steps(lambda: s.step(dt, c, w), steps))
    s.stats(reset=True)
    R.rmhd_set_timing(s.ctx, True)
    R.rmhd_get_timing(s.ctx, reset=True)
    for _ in range(timing_steps):
        s.step(dt, c, w)
    tm = R.rmhd_get_timing(s.ctx, reset=True)
    st2 = s.stats(reset=True)
    R.rmhd_set_timing(s.ctx, False)
    s.set_stats_detail(True)
    for _ in range(2):
        s.step(dt, c, w)
    sd = s.stats(reset=True)
    s.close()
    out = {"cells": wl.cells, "steps": steps, "ms_per_step": ms[0], "value": wl.cells / (ms[0] / 1e3),
           "unit": "cell-updates/s", "ms_per_step_runs": ms, "value_median": wl.cells / (sorted(ms)[len(ms) // 2] / 1e3)}
    if wl.model != 2:
        out.update(newton_fields(R, st, sd))
    stage_ms = tm["stage_ms"] / tm["stage_launches"] if tm["stage_launches"] else None
    flux_ms = tm["flux_ms"] / tm["flux_launches"]
    out["kernels"] = {"flux_ms_per_pass": flux_ms, "stage_ms_per_launch": stage_ms,
                      "c2p_ms_per_launch": tm["c2p_ms"] / tm["c2p_launches"] if tm["c2p_launches"] else None}
    if stage_ms is not None:
        flops = PM.stage_flops_of(wl.model, st2) / tm["stage_launches"]
        tf = flops / (stage_ms / 1e3) / 1e12
        out["kernels"]["stage"] = {"bound": "alu", "achieved": tf, "peak": PM.PEAK_FP64_VECTOR_TFLOPS,
                                   "unit": "TFLOP/s", "frac": tf / PM.PEAK_FP64_VECTOR_TFLOPS,
                                   "flops_per_launch": flops,
                                   "flops_per_cell": PM.stage_flops_of(wl.model, st2) / max(1, st2["stage_cells"]),
                                   "ms_per_launch": stage_ms}
    fb = 0.5 * (PM.flux_bytes_per_cell(wl.model, "first") + PM.flux_bytes_per_cell(wl.model, "second"))
    if tm["c2p_launches"]:   # the new primitives come from a separate recovery kernel
        fb -= 0.5 * 8 * PM.NPRIM[wl.model]
    gbs = fb * wl.cells / (flux_ms / 1e3) / 1e9
    out["kernels"]["flux"] = {"bound": "hbm", "achieved": gbs, "peak": PM.PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": gbs / PM.PEAK_HBM_GBS, "bytes_per_cell": fb,
                              "bytes_per_launch": fb * wl.cells, "ms_per_launch": flux_ms}
    return out


def batched_measure(steps: int, warmup: int) -> dict:
    """The 64-domain batched workload (32 1-D shock tubes, N ~ U[128, 4096]; 32 2-D KH set-ups,
    sides ~ U[64, 512]; sigma ~ 10^U[1, 6]; seed 4): the autotuned batched step; the same
    shape with the stage queue and with the persistent stage launch switched on and off; and
    the same domains stepped one after another on the single-grid path, launched directly and
    replayed from one HIP graph per domain."""
    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL
    doms = WL.batched_domains(seed=4)
    cells = sum(w.cells for w in doms)
    B = R.Batch(doms)
    tuning = B.autotune()
    for _ in range(warmup):
        B.step()
    B.stats(reset=True)
    ms_b = timed_steps(B.step, steps)
    st = B.stats(reset=True)
    B.set_stats_detail(True)          # one untimed step for the step-count histogram
    B.step()
    sd = B.stats(reset=True)
    B.set_stats_detail(False)
    variants = {}
    base = {k: tuning[k] for k in ("persistent", "chunks_per_item", "persistent_blocks", "newton_cap", "flux_rows",
                                   "use_graph")}
    for name, kw in (("queue_after_2", {"newton_cap": 2}), ("queue_after_3", {"newton_cap": 3}),
                     ("no_queue", {"newton_cap": 50}), ("persistent", {"persistent": 1}),
                     ("one_block_per_item", {"persistent": 0}), ("no_graph", {"use_graph": 0})):
        B.tune(**{**base, **kw})
        for _ in range(2):
            B.step()
        variants[name] = timed_steps(B.step, steps)
    B.tune(**base)
    B.close()
    per_domain = {}
    for graph in (False, True):
        solvers = []
        for wl in doms:
            s = R.Solver(R.params_from(wl))
            c, w = s.initial_state(wl.prims, wl.EB)
            if graph:
                s.set_graph(True)
            solvers.append((s, c, w, s.dt()))

        def step_all():
            for s, c, w, h in solvers:
                s.step(h, c, w)
        for _ in range(warmup):
            step_all()
        per_domain["graph" if graph else "direct"] = timed_steps(step_all, steps)
        for s, *_ in solvers:
            s.close()
    return {"workload": "64 domains (32 x 1-D Brio-Wu N~U[128,4096], 32 x 2-D KHI sides~U[64,512], "
                        "sigma~10^U[1,6], seed 4)", "cells": cells,
            "value": cells / (ms_b / 1e3), "unit": "cell-updates/s", "ms_per_step": ms_b,
            "tuning": tuning, **newton_fields(R, st, sd),
            "variants_ms_per_step": variants,
            "per_domain_ms_per_step": per_domain,
            "speedup_vs_per_domain_direct": per_domain["direct"] / ms_b,
            "speedup_vs_per_domain_graph": per_domain["graph"] / ms_b}


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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--timing-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="headline workload only")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ssp3", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-ideal", action="store_true")
    ap.add_argument("--only-3d", action="store_true",
                    help="print the 3-D grid measurements alone (for profiling the 3-D flux pass)")
    ap.add_argument("--only-batched", action="store_true",
                    help="time the 64-domain batched step alone at the autotuner's usual shape (one block "
                         "per stage item, no queue, HIP graph), without tuning runs, for profiling")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (traffic calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU form would shard the grid into slabs with a halo exchange per flux pass; it is not built)",
              file=sys.stderr)
        return 2

    import torch

    from paper_1808_09721_amd import rmhd as R
    from paper_1808_09721_amd import workloads as WL

    torch.cuda.set_device(0)
    R.lib()
    if args.only_3d:
        copy_calibration(args.copy_mib)
        print(json.dumps({"grid3d": grid3d_measure(max(3, args.steps // 20), args.warmup)}), flush=True)
        return 0
    if args.only_batched:
        copy_calibration(args.copy_mib)
        doms = WL.batched_domains(seed=4)
        B = R.Batch(doms)
        B.tune(persistent=0, newton_cap=50, flux_rows=16, use_graph=1)
        for _ in range(args.warmup):
            B.step()
        ms = timed_steps(B.step, args.steps)
        B.close()
        cells = sum(w.cells for w in doms)
        print(json.dumps({"batched": {"cells": cells, "ms_per_step": ms, "value": cells / (ms / 1e3),
                                      "unit": "cell-updates/s"}}), flush=True)
        return 0
    wall0 = time.perf_counter()
    # the network, trained on the device on rows harvested from 512^2 sheets at seeds 1-4
    # (outside every timed region)
    net, training = R.train_guess_network()
    wl = WL.learned_guess_sheet(1024, seed=5, steps=args.steps)
    plain = measure_form(wl, args.steps, args.warmup, timing_steps=args.timing_steps)
    learned = measure_form(wl, args.steps, args.warmup, timing_steps=args.timing_steps, net=net)
    wall = time.perf_counter() - wall0
    copy_calibration(args.copy_mib)
    k = plain["kernels"]
    dominant = "stage" if k["stage"]["ms_per_launch"] >= k["flux"]["ms_per_launch"] else "flux"
    roof = {kk: k[dominant][kk] for kk in ("bound", "achieved", "peak", "unit", "frac")}
    roof["kernel"] = "implicit stage k_stage<1>" if dominant == "stage" else "flux pass k_flux<1, 2, 64, 12, *>"
    roof["traffic"] = measured_traffic("two_fluid_sheet_1024",
                                       "rmhd::k_stage<1>" if dominant == "stage" else "rmhd::k_flux<1, 2")
    value = plain["value"]
    out = {
        "metric": "FP64 cell-updates/s per IMEX step + Newton iters/cell, plain vs batched+learned",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": plain["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "two-fluid current sheet 1024x1024 periodic, mu=+-1000, Gamma=4/3, sigma~10^U[2,6] "
                               "per cell, seed 5, SSP2(222) IMEX + FVS/WENO3, FP64 Newton to 1e-12 per cell; "
                               "plain form (learned form in 'learned')",
                   "cells": wl.cells, "parallelism": "single GPU"},
        "value_median_of_5": plain["value_median"],
        "ms_per_step_runs": plain["ms_per_step_runs"],
        "newton_iters_per_cell_stage": plain["newton_iters_per_cell_stage"],
        "roofline": roof,
        "plain": plain,
        "learned": learned,
        "learned_speedup_vs_plain": plain["ms_per_step"] / learned["ms_per_step"],
        "training": training,
        "wall_s": wall,
    }
    net.close()
    if not args.no_secondary:
        khi = measure_form(WL.kelvin_helmholtz_2d(), args.steps, args.warmup, timing_steps=args.timing_steps)
        t = measured_traffic("khi_256x512", "rmhd::k_flux<0, 2, 64, 16")
        khi["kernels"]["flux"]["traffic"] = t
        out["kelvin_helmholtz_256x512"] = khi
        bw = WL.brio_wu_1d(400)
        out["brio_wu_400"] = measure_form(bw, 320, args.warmup, runs=3, timing_steps=args.timing_steps)
        out["brio_wu_400"]["note"] = "320 steps of dt = CFL dx (t = 0.4) per timed region"
        out["two_fluid_sheet_512"] = measure_form(WL.two_fluid_sheet_2d(512, 512), args.steps, args.warmup, runs=3,
                                                  timing_steps=args.timing_steps)
        if not args.no_batched:
            out["batched"] = batched_measure(max(5, args.steps // 5), args.warmup)
        if not args.no_ssp3:
            out["ssp3"] = ssp3_measure(max(10, args.steps // 2), args.warmup)
        if not args.no_3d:
            out["grid3d"] = grid3d_measure(max(3, args.steps // 20), args.warmup)
        if not args.no_ideal:
            out["ideal"] = ideal_measure(max(10, args.steps // 2), args.warmup, khi["ms_per_step"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["gpu_speedup"] = value / out["cpu_baseline"]["value"]
        out["cpu_baseline"]["single_core"]["gpu_speedup"] = value / out["cpu_baseline"]["single_core"]["value"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
