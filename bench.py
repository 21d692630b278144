#!/usr/bin/env python3
"""Benchmark: time steps/s of ROM-accelerated SI-DSA vs plain SI-DSA at 1e-8
relative tolerance on one MI355X, printed as one JSON line.

A "step" is one backward-Euler time step of the whole hot path: initial guess,
source iterations with sweeps + moments + DSA / ROM correction, final f and
right-hand-side sweeps, and the ROM bookkeeping.  Inputs are synthetic and
seeded (paper_2603_19647_amd.workloads) and resident on the device before the
timed region starts.

Workloads:
  slab4096  4096-cell slab, 64-point Gauss-Legendre, 32 random regions,
            dt = 0.005; ROM-SI-DSA with FP32 sweeps + FP64 refinement vs
            SI-DSA with the same kernels and precision.
  batch512  512 independent slabs (128..2048 cells, S_16/32/64, 8 regions),
            dt = 0.01, fused into shared launches; value in instance-steps/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector; non-packed FP32 issues at the same lane rate
SLAB_SWEEP_FLOPS = 6         # per cell-angle update: 2 mul, 2 fma-equivalent, 1 add, 1 division
FPASS_BYTES_PER_CELL_ANGLE = 16   # f^{n-1} read + f^n write, FP64
FPASS_BYTES_PER_CELL = 7 * 8      # sigma_t~, sigma_s, G, rho^n, b~ read; b~, b~_prev write


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def run_single(spec, warmup, steps, rtrom):
    if warmup > 0:
        w = rtrom.Problem(spec)
        w.march(warmup)
        w.close()
    p = rtrom.Problem(spec)
    sync()
    rtrom.profile_enable(True)
    t0 = time.perf_counter()
    p.march(steps)
    sync()
    t1 = time.perf_counter()
    prof = rtrom.profile_read()
    rtrom.profile_enable(False)
    st = p.stats()
    p.close()
    return t1 - t0, st, prof


def run_batch(specs, warmup, steps, rtrom):
    if warmup > 0:
        ws = [rtrom.Problem(s) for s in specs[:64]]
        rtrom.march_batch(ws, warmup)
        for w in ws:
            w.close()
    probs = [rtrom.Problem(s) for s in specs]
    sync()
    rtrom.profile_enable(True)
    t0 = time.perf_counter()
    rtrom.march_batch(probs, steps)
    sync()
    t1 = time.perf_counter()
    prof = rtrom.profile_read()
    rtrom.profile_enable(False)
    stats = [p.stats() for p in probs]
    for p in probs:
        p.close()
    return t1 - t0, stats, prof


def roofline(prof, si_updates, fpass_cell_angles, fpass_cells):
    """Achieved rate of the dominant kernel against its bound."""
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    sec, launches = kinds[dom]
    avg = sec / launches
    if dom == "slab_fpass":
        traffic_b = FPASS_BYTES_PER_CELL_ANGLE * fpass_cell_angles + FPASS_BYTES_PER_CELL * fpass_cells
        ach = traffic_b / sec / 1e9
        return dom, avg, {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": ach / HBM_PEAK_GBS, "traffic": None}
    if dom == "slab_si":
        flops = SLAB_SWEEP_FLOPS * si_updates
        ach = flops / sec / 1e12
        return dom, avg, {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / FP64_VECTOR_TFLOPS, "traffic": None}
    return dom, avg, {"bound": "alu", "achieved": None, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                      "frac": None, "traffic": None}


def cpu_baseline_slab(spec, seconds_budget=20.0):
    """The FP64 oracle (ROM-SI-DSA) on the host, one core, a bounded number of steps."""
    import oracle
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    n, t0 = 0, time.perf_counter()
    while n < spec.nsteps and time.perf_counter() - t0 < seconds_budget:
        o.step()
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "time steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} steps of the same problem, FP64 oracle, single thread"}


def _oracle_instance(args):
    spec, steps = args
    import oracle
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    o.march(steps)
    return steps


def cpu_baseline_batch(specs, steps, seconds_budget=20.0):
    import multiprocessing as mp
    cores = min(16, os.cpu_count() or 1)
    sample = specs[: max(cores, 1) * 2]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        done = sum(pool.map(_oracle_instance, [(s, steps) for s in sample]))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "instance-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} of the 512 instances x {steps} steps, FP64 oracle, process pool"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=("slab4096", "batch512"), default="slab4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    from paper_2603_19647_amd import rtrom
    from paper_2603_19647_amd import workloads as W

    if args.workload == "slab4096":
        spec = W.slab_random_regions()
        steps = spec.nsteps if args.steps is None else args.steps
        warm = 20 if args.warmup is None else args.warmup
        spec = spec.replace(nsteps=steps)
        nc, nv = spec.ncells, spec.nord
        log(f"bench: slab4096 ROM mixed, {steps} steps")
        t_rom, st_rom, prof_rom = run_single(spec, warm, steps, rtrom)
        log(f"bench: slab4096 SI-DSA mixed, {steps} steps")
        t_si, st_si, prof_si = run_single(spec.replace(method="si_dsa"), warm, steps, rtrom)
        value = steps / t_rom
        si_val = steps / t_si
        updates = st_rom["sweeps_total"] * nc * nv
        dom, avg, roof = roofline(prof_rom, st_rom["si_iters_total"] * nc * nv, steps * nc * nv, steps * nc)
        extra = {
            "si_dsa_steps_per_s": si_val,
            "speedup_vs_si_dsa": value / si_val,
            "cell_angle_updates_per_s": updates / t_rom,
            "si_dsa_cell_angle_updates_per_s": st_si["sweeps_total"] * nc * nv / t_si,
            "si_sweeps_per_step": st_rom["si_iters_total"] / steps,
            "si_dsa_si_sweeps_per_step": st_si["si_iters_total"] / steps,
            "fp32_sweeps": st_rom["fp32_sweeps"], "n0": st_rom["n0"], "n1": st_rom["n1"],
            "kernel_ms": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof_rom.items() if v[1]},
            "si_dsa_kernel_ms": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof_si.items() if v[1]},
        }
        config = {"workload": "slab4096_gl64_32regions", "cells": nc, "ordinates": nv, "dt": spec.dt,
                  "tol": spec.tol, "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refine",
                  "baseline_method": "si_dsa (same kernels and precision)", "instances": 1}
        metric = "time steps/s (ROM-SI-DSA, 1e-8 rel tol)"
        unit = "steps/s"
        cpu = None if args.no_cpu_baseline else cpu_baseline_slab(spec)
    else:
        specs = W.slab_batch()
        steps = specs[0].nsteps if args.steps is None else args.steps
        warm = 5 if args.warmup is None else args.warmup
        log(f"bench: batch512 ROM mixed, {steps} steps")
        t_rom, sts, prof_rom = run_batch(specs, warm, steps, rtrom)
        log(f"bench: batch512 SI-DSA mixed, {steps} steps")
        t_si, sts_si, prof_si = run_batch([s.replace(method="si_dsa") for s in specs], warm, steps, rtrom)
        n = len(specs)
        value = n * steps / t_rom
        si_val = n * steps / t_si
        ca = [s.ncells * s.nord for s in specs]
        upd = sum(st["sweeps_total"] * c for st, c in zip(sts, ca))
        si_upd = sum(st["si_iters_total"] * c for st, c in zip(sts, ca))
        dom, avg, roof = roofline(prof_rom, si_upd, steps * sum(ca), steps * sum(s.ncells for s in specs))
        extra = {
            "si_dsa_instance_steps_per_s": si_val,
            "speedup_vs_si_dsa": value / si_val,
            "cell_angle_updates_per_s": upd / t_rom,
            "si_sweeps_per_step": sum(st["si_iters_total"] for st in sts) / (n * steps),
            "si_dsa_si_sweeps_per_step": sum(st["si_iters_total"] for st in sts_si) / (n * steps),
            "kernel_ms": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof_rom.items() if v[1]},
            "si_dsa_kernel_ms": {k: (v[0] / v[1] * 1e3 if v[1] else None) for k, v in prof_si.items() if v[1]},
        }
        config = {"workload": "batch512_slabs", "instances": n, "steps_each": steps,
                  "cells": "128..2048", "ordinates": "16/32/64", "dt": 0.01, "tol": 1e-8,
                  "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refine",
                  "baseline_method": "si_dsa (same kernels and precision)"}
        metric = "instance time steps/s (ROM-SI-DSA, 1e-8 rel tol)"
        unit = "instance-steps/s"
        cpu = None if args.no_cpu_baseline else cpu_baseline_batch(specs, steps)

    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg * 1e3
    out = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": t_rom / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": config, "roofline": roof, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
