#!/usr/bin/env python3
"""Benchmark: time steps/s of ROM-accelerated SI-DSA against plain SI-DSA at a
1e-8 relative tolerance on one MI355X, printed as one JSON line.

A "step" is one backward-Euler time step of the whole hot path: initial
guess, source iterations (sweeps + moments + DSA / ROM correction), the final
f and right-hand-side sweeps, and the ROM bookkeeping (snapshots, incremental
SVD, DMD operators).  Inputs are synthetic and seeded
(paper_2603_19647_amd.workloads) and resident on the device before the timed
region starts.  Both methods run the same kernels at the same precision
(FP32 sweeps refined by FP64 sweeps, FP64 everything else).

Workloads (--workload):
  slab4096    4096-cell slab, 64-point Gauss-Legendre, 32 seeded regions,
              dt = 0.005, 400 steps (default).
  checker256  256 x 256 checkerboard, CL(16, 8) = 128 directions, dt = 0.01,
              200 steps.
  batch512    512 independent slabs (128..2048 cells, S_16/32/64, 8 regions),
              dt = 0.01, 100 steps each, fused launches; instance-steps/s.
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

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
VALU_PEAK_TFLOPS = 78.6     # MI355X FP64 vector; FP32 without packed math issues at the same lane rate
# algorithmic FLOPs of one cell-angle update of an upwind sweep plus its
# moment accumulation: 1D  f = (s + m f_in) / (ct + m), rho += w f
#                       2D  f = (s + mx f_l + my f_b) / (ct + mx + my), rho += w f
SWEEP_FLOPS = {1: 6, 2: 8}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_single(spec, warmup, steps, rtrom):
    if warmup > 0:
        w = rtrom.Problem(spec)
        w.march(warmup)
        w.close()
    p = rtrom.Problem(spec)
    p.march(0)
    rtrom.profile_enable(True)
    t0 = time.perf_counter()
    p.march(steps)          # returns after the device finished the march
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
    rtrom.profile_enable(True)
    t0 = time.perf_counter()
    rtrom.march_batch(probs, steps)
    t1 = time.perf_counter()
    prof = rtrom.profile_read()
    rtrom.profile_enable(False)
    stats = [p.stats() for p in probs]
    for p in probs:
        p.close()
    return t1 - t0, stats, prof


def copy_probe(mib: int):
    """A plain device-to-device copy of known size (read and write mib MiB each
    time), for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"bench: copy probe {mib} MiB x 5")


# Sources of the dominant kernels: a stored counter measurement is used only
# while these files are unchanged.
KERNEL_SOURCES = {
    "k_si_slab": ["rt_slab.hip", "rt_common.h", "rt_rom.h", "rt_arrow.h", "rt_capi.hip"],
    "k_plane_sweep": ["rt_plane.hip", "rt_common.h"],
}


def sources_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2603_19647_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from profiles/<kernel>_<workload>_traffic.md (two
    rocprofv3 --pmc runs, FETCH_SIZE and WRITE_SIZE, scaled by the same
    counters on a copy of known size), or None when absent or when the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    digest, value = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("sources sha256:"):
                digest = line.split(":", 1)[1].strip()
            if line.startswith("HBM bytes per dispatch:"):
                value = float(line.split(":", 1)[1].strip())
    return value if digest == sources_digest(kernel) and value is not None else None


def kernel_ms(prof):
    return {k: v[0] / v[1] * 1e3 for k, v in prof.items() if v[1]}


def roofline_sweep(prof, kind, dim, updates, kernel):
    """The dominant kernel is a sweep-bound kernel: FLOP rate of its cell-angle
    updates (algorithmic FLOPs / event-timed launch duration) against the
    vector ALU peak."""
    sec, launches = prof[kind]
    flops = SWEEP_FLOPS[dim] * updates
    ach = flops / sec / 1e12
    return {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / VALU_PEAK_TFLOPS, "traffic": None, "kernel": kernel, "kind": kind,
            "launches": launches, "avg_launch_ms": sec / launches * 1e3,
            "flops_per_launch": flops / launches}


def roofline_dsa(prof, nc, cheb_iters):
    """Chebyshev DSA solve: algorithmic bytes of the unfused iteration (read
    d, r, x, diag, ax, ay; write d, r, x: 9 doubles per cell) per iteration."""
    sec, launches = prof["plane_dsa"]
    bytes_ = 72.0 * nc * cheb_iters * launches
    ach = bytes_ / sec / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "k_dsa_block", "kind": "plane_dsa",
            "launches": launches, "avg_launch_ms": sec / launches * 1e3,
            "bytes_per_launch": bytes_ / launches}


def cpu_baseline_single(spec, seconds_budget=20.0):
    """The FP64 oracle (same method) on the host, one core, the first steps of
    the same problem within a time budget."""
    import oracle
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    n, t0 = 0, time.perf_counter()
    while n < spec.nsteps and time.perf_counter() - t0 < seconds_budget:
        o.step()
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {spec.nsteps} steps of the same problem, FP64 oracle, one thread"}


def _oracle_instance(args):
    spec, steps = args
    import oracle
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    o.march(steps)
    return steps


def cpu_baseline_batch(specs, steps, seconds_budget=20.0):
    import multiprocessing as mp
    cores = min(16, os.cpu_count() or 1)
    sample = specs[: cores * 2]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        done = sum(pool.map(_oracle_instance, [(s, steps) for s in sample]))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "instance-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} of the {len(specs)} instances x {steps} steps, FP64 oracle, process pool"}


def run_serving(rtrom, W, count, budget, slots, seed=5):
    """C5: closed-loop saturation run (everything submitted at once) gives the
    capacity; then Poisson arrivals at 80 % of it, with per-step and per-march
    latencies and the queueing delay seen by the client."""
    import numpy as np
    specs = W.serving_stream(seed=seed, count=count)
    # closed loop
    srv = rtrom.Server(hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()
    tickets = [srv.submit(s) for s in specs]
    srv.drain()
    t_sat = time.perf_counter() - t0
    for t in tickets:
        srv.fetch(t)
    srv.close()
    steps_total = sum(s.nsteps for s in specs)
    capacity = count / t_sat
    # open loop, Poisson arrivals at 0.8 x capacity
    rng = np.random.default_rng(seed + 1000)
    gaps = rng.exponential(1.0 / (0.8 * capacity), size=count)
    srv = rtrom.Server(hbm_budget_bytes=budget, max_slots=slots)
    sub_t, done_t, tickets = {}, {}, []
    t0 = time.perf_counter()
    nxt = 0
    arrive = t0 + np.cumsum(gaps)
    while len(done_t) < count:
        now = time.perf_counter()
        while nxt < count and arrive[nxt] <= now:
            tk = srv.submit(specs[nxt])
            tickets.append(tk)
            sub_t[tk] = now
            nxt += 1
        for tk in tickets:
            if tk not in done_t and srv.poll(tk) >= 2:
                done_t[tk] = time.perf_counter()
        time.sleep(0.0005)
    t_open = time.perf_counter() - t0
    step_lat, march_lat, e2e = [], [], []
    for tk in tickets:
        rho, st, lat, mlat = srv.fetch(tk)
        step_lat.extend(lat.tolist())
        march_lat.append(mlat)
        e2e.append(done_t[tk] - sub_t[tk])
    srv.close()
    p = lambda a, q: float(np.percentile(np.asarray(a), q))
    return {
        "requests": count, "instance_steps": steps_total, "saturation_s": t_sat,
        "capacity_requests_per_s": capacity, "saturation_instance_steps_per_s": steps_total / t_sat,
        "open_loop_rate_requests_per_s": 0.8 * capacity, "open_loop_s": t_open,
        "open_loop_instance_steps_per_s": steps_total / t_open,
        "step_latency_ms": {"p50": p(step_lat, 50) * 1e3, "p99": p(step_lat, 99) * 1e3},
        "march_latency_s": {"p50": p(march_lat, 50), "p99": p(march_lat, 99)},
        "end_to_end_latency_s": {"p50": p(e2e, 50), "p99": p(e2e, 99)},
        "hbm_budget_bytes": budget, "max_slots": slots,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=("slab4096", "checker256", "batch512", "serving"), default="slab4096")
    ap.add_argument("--requests", type=int, default=24, help="serving: requests in the stream")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serving: HBM admission budget")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent problems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device five times (a plain copy of known size, "
                         "against which hardware byte counters are scaled)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(each problem, or each instance of a batch, runs on one device)", file=sys.stderr)
        sys.exit(2)

    from paper_2603_19647_amd import rtrom
    from paper_2603_19647_amd import workloads as W

    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    extra = {}
    if args.workload in ("slab4096", "checker256"):
        spec = W.slab_random_regions() if args.workload == "slab4096" else W.checkerboard()
        steps = spec.nsteps if args.steps is None else args.steps
        warm = (20 if args.workload == "slab4096" else 5) if args.warmup is None else args.warmup
        spec = spec.replace(nsteps=steps)
        nc, nv = spec.ncells, spec.nord
        log(f"bench: {args.workload} ROM-SI-DSA mixed, {steps} steps")
        t_rom, st_rom, prof_rom = run_single(spec, warm, steps, rtrom)
        log(f"bench: {args.workload} SI-DSA mixed, {steps} steps")
        t_si, st_si, prof_si = run_single(spec.replace(method="si_dsa"), warm, steps, rtrom)
        value = steps / t_rom
        si_val = steps / t_si
        nfold = nv if spec.dim == 1 else nv // 2   # 2D sweeps the Omega_z > 0 half
        if spec.dim == 1:
            roof = roofline_sweep(prof_rom, "slab_si", 1, st_rom["si_iters_total"] * nc * nv,
                                  "k_si_slab")
        else:
            kinds = {k: v[0] for k, v in prof_rom.items() if v[1]}
            if max(kinds, key=kinds.get) == "plane_dsa":
                roof = roofline_dsa(prof_rom, nc, st_rom["dsa_iters"])
            else:
                roof = roofline_sweep(prof_rom, "plane_sweep", 2, st_rom["si_iters_total"] * nc * nfold,
                                      "k_plane_sweep")
        extra = {
            "si_dsa_steps_per_s": si_val,
            "speedup_vs_si_dsa": value / si_val,
            "cell_angle_updates_per_s": st_rom["sweeps_total"] * nc * nv / t_rom,
            "si_sweeps_per_step": st_rom["si_iters_total"] / steps,
            "si_dsa_si_sweeps_per_step": st_si["si_iters_total"] / steps,
            "fp32_sweeps": st_rom["fp32_sweeps"], "n0": st_rom["n0"], "n1": st_rom["n1"],
            "rank_ig": st_rom["rank_ig"], "rank_pc": st_rom["rank_pc"],
            "nonconverged_steps": st_rom["nonconverged_steps"],
            "kernel_ms": kernel_ms(prof_rom), "si_dsa_kernel_ms": kernel_ms(prof_si),
        }
        if spec.dim == 1:
            config = {"workload": "slab4096_gl64_32regions", "cells": nc, "ordinates": nv, "dt": spec.dt,
                      "steps": steps, "tol": spec.tol}
        else:
            config = {"workload": "checkerboard256_cl16x8", "cells": nc, "ordinates": nv, "dt": spec.dt,
                      "steps": steps, "tol": spec.tol}
        config.update({"method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refinement",
                       "baseline_method": "si_dsa, same kernels and precision", "instances": 1})
        metric = "time steps/s (ROM-SI-DSA, 1e-8 rel tol)"
        unit = "steps/s"
        cpu = None if args.no_cpu_baseline else cpu_baseline_single(spec)
    elif args.workload == "serving":
        # Disabled: a serving run on the GPU completed and printed its line,
        # but the process then crashed during exit (status 139) with the cause
        # not established; the serving tests under pytest pass.
        print("bench.py: the serving workload is disabled until a crash at process exit "
              "after the serving run is explained", file=sys.stderr)
        sys.exit(3)
        warm = 0
        log(f"bench: serving stream of {args.requests} requests")
        res = run_serving(rtrom, W, args.requests, int(args.budget_gib * (1 << 30)), args.slots)
        steps = res["instance_steps"]
        value = res["saturation_instance_steps_per_s"]
        t_rom = res["saturation_s"]
        roof = None
        extra = {"serving": res}
        config = {"workload": "serving_stream_grf_2d", "requests": args.requests,
                  "grids": "64..512 squared", "ordinates": "32/64/128", "steps_each": "100..500",
                  "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refinement",
                  "arrivals": "closed loop (value), then Poisson at 0.8 x capacity"}
        metric = "instance time steps/s, serving (ROM-SI-DSA, 1e-8 rel tol)"
        unit = "instance-steps/s"
        cpu = None
    else:
        specs = W.slab_batch()
        steps = specs[0].nsteps if args.steps is None else args.steps
        warm = 5 if args.warmup is None else args.warmup
        log(f"bench: batch512 ROM-SI-DSA mixed, {steps} steps")
        t_rom, sts, prof_rom = run_batch(specs, warm, steps, rtrom)
        log(f"bench: batch512 SI-DSA mixed, {steps} steps")
        t_si, sts_si, prof_si = run_batch([s.replace(method="si_dsa") for s in specs], warm, steps, rtrom)
        n = len(specs)
        value = n * steps / t_rom
        si_val = n * steps / t_si
        ca = [s.ncells * s.nord for s in specs]
        si_upd = sum(st["si_iters_total"] * c for st, c in zip(sts, ca))
        roof = roofline_sweep(prof_rom, "slab_si", 1, si_upd, "k_si_slab")
        extra = {
            "si_dsa_instance_steps_per_s": si_val,
            "speedup_vs_si_dsa": value / si_val,
            "cell_angle_updates_per_s": sum(st["sweeps_total"] * c for st, c in zip(sts, ca)) / t_rom,
            "si_sweeps_per_step": sum(st["si_iters_total"] for st in sts) / (n * steps),
            "si_dsa_si_sweeps_per_step": sum(st["si_iters_total"] for st in sts_si) / (n * steps),
            "kernel_ms": kernel_ms(prof_rom), "si_dsa_kernel_ms": kernel_ms(prof_si),
        }
        config = {"workload": "batch512_slabs", "instances": n, "steps": steps,
                  "cells": "128..2048", "ordinates": "16/32/64", "dt": 0.01, "tol": 1e-8,
                  "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refinement",
                  "baseline_method": "si_dsa, same kernels and precision"}
        metric = "instance time steps/s (ROM-SI-DSA, 1e-8 rel tol)"
        unit = "instance-steps/s"
        cpu = None if args.no_cpu_baseline else cpu_baseline_batch(specs, steps)

    if roof is not None:
        wl_name = {"slab4096_gl64_32regions": "slab4096", "checkerboard256_cl16x8": "checker256",
                   "batch512_slabs": "batch512"}.get(config.get("workload"), "")
        roof["traffic"] = stored_traffic(roof["kernel"], wl_name)
    out = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": t_rom / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": config, "roofline": roof, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
