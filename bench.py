#!/usr/bin/env python3
"""Benchmark: time steps/s of ROM-accelerated SI-DSA against plain SI-DSA at a
1e-8 relative tolerance on one MI355X, printed as one JSON line.

A "step" is one backward-Euler time step of the whole hot path for every
instance of the workload: initial guess, source iterations (sweeps + moments
+ DSA / ROM correction), the final f and right-hand-side sweeps, and the ROM
bookkeeping (snapshots, incremental SVD, DMD operators).  Inputs are synthetic
and seeded (paper_2603_19647_amd.workloads) and resident on the device before
the timed region starts.  Both methods run the same kernels at the same
precision (FP32 sweeps refined by FP64 sweeps, FP64 everything else).

The W warmup steps are the first W steps of the same march (untimed); the K
timed steps follow them.  A "full_march" block times, on fresh problems, the
whole configured march of each method (phases I-III inside the timed value).

Workloads (--workload):
  batch512    512 independent slabs (128..2048 cells, S_16/32/64, 8 regions),
              dt = 0.01, 100 steps each, fused launches; instance-steps/s
              (default: the largest single-GPU workload).
  slab4096    4096-cell slab, 64-point Gauss-Legendre, 32 seeded regions,
              dt = 0.005, 400 steps.
  checker256  256 x 256 checkerboard, CL(16, 8) = 128 directions, dt = 0.01,
              200 steps.
  serving     stream of 2D requests (grids 64..512 squared, 32..128
              directions, 100..500 steps): closed-loop capacity, then Poisson
              arrivals at 80 % of it with per-step, per-march and end-to-end
              latency percentiles.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
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
# 1D piecewise-linear DG: per cell-angle the 2x2 upwind solve (determinant,
# two right-hand sides, two unknowns), the outflow value and two moment
# updates, 22 FLOPs, i.e. 11 per unknown-angle update
SWEEP_FLOPS_DG1 = 11
# algorithmic HBM bytes (FP64):
FPASS_BYTES_PER_CELL_ANGLE = 16   # f^{n-1} read, f^n written
FPASS_BYTES_PER_CELL = 40         # sigma_t, sigma_s, rho^n, G read; b~^n written
SI_BYTES_PER_CELL = 80            # per step: sigma_t, sigma_s, b~, rho^{n-1}, three DSA factors read;
                                  # rho^n, rho^(1/2) and the initial guess written
ROM_BYTES_PER_CELL_COLUMN = 56    # per update and basis column: the two Gram-Schmidt passes read U, then
                                  # U and W (App. B, CGS applied twice); the rotation reads and writes U and W


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def kernel_ms(prof):
    return {k: v[0] / v[1] * 1e3 for k, v in prof.items() if v[1]}


def kernel_table(prof, fpass_bytes, si_bytes, rom_bytes):
    """Per kernel kind: launches, mean duration (HIP events on the launch's
    stream) and algorithmic HBM GB/s against the 8 TB/s peak."""
    out = {}
    for kind, nbytes in (("slab_fpass", fpass_bytes), ("slab_si", si_bytes), ("post", rom_bytes)):
        sec, n = prof.get(kind, (0.0, 0))
        if not n:
            continue
        gbs = nbytes / sec / 1e9 if sec > 0 else 0.0
        out[kind] = {"launches": n, "avg_launch_ms": sec / n * 1e3, "algorithmic_bytes_per_launch": nbytes / n,
                     "achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        if kind == "post":  # second stream: the events also bracket the wait for compute units
            out[kind]["timing"] = "event pair includes the wait for compute units beside the f-pass"

    return out


def roofline_sweep(prof, kind, dim, updates, kernel, flops_per_update=None):
    """The SI sweep kernel is bound by the vector ALU: FLOP rate of its
    cell-angle updates (algorithmic FLOPs / event-timed launch duration)
    against the FP64 vector peak."""
    sec, launches = prof[kind]
    flops = (SWEEP_FLOPS[dim] if flops_per_update is None else flops_per_update) * updates
    ach = flops / sec / 1e12
    return {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / VALU_PEAK_TFLOPS, "traffic": None, "kernel": kernel, "kind": kind,
            "launches": launches, "avg_launch_ms": sec / launches * 1e3,
            "flops_per_launch": flops / launches}


def roofline_hbm(prof, kind, nbytes, kernel):
    """An HBM-bound kernel: algorithmic bytes of its launches / their
    event-timed duration, against the 8 TB/s peak."""
    sec, launches = prof[kind]
    ach = nbytes / sec / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernel, "kind": kind, "launches": launches,
            "avg_launch_ms": sec / launches * 1e3, "bytes_per_launch": nbytes / launches}


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


# Sources of the dominant kernels: a stored counter measurement is used only
# while these files are unchanged.
KERNEL_SOURCES = {
    "k_si_slab": ["rt_slab.hip", "rt_common.h", "rt_rom.h", "rt_arrow.h", "rt_capi.hip"],
    "k_si_wave": ["rt_wave.hip", "rt_common.h", "rt_rom.h", "rt_dsa.h", "rt_mh.h", "rt_arrow.h"],
    "k_fpass_wave": ["rt_wave.hip", "rt_common.h"],
    "k_fpass_dg": ["rt_wave.hip", "rt_common.h"],
    "k_rom_post_small": ["rt_rom.hip", "rt_rom.h", "rt_arrow.h", "rt_common.h"],
    "k_plane_sweep": ["rt_plane.hip", "rt_common.h"],
}


def sources_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_2603_19647_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per dispatch from profiles/<kernel>_<workload>_traffic.md (two
    rocprofv3 --pmc runs, FETCH_SIZE and WRITE_SIZE, scaled by the same
    counters on a copy of known size), or None when absent or when the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
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


# --------------------------------------------------------------------------
# marches
# --------------------------------------------------------------------------

def timed_batch(rtrom, specs, warmup, steps, profile=True):
    """Create the problems, march `warmup` steps untimed, then time `steps`
    further steps of the same march (fused launches over all instances, the
    step replayed from a HIP graph).  With `profile`, a second set of the same
    problems marches the same window again with every launch bracketed by
    events (eagerly), for the per-kernel durations; the march is
    deterministic, so both windows do the same work."""
    probs = [rtrom.Problem(s) for s in specs]
    if warmup > 0:
        rtrom.march_batch(probs, warmup)
    t0 = time.perf_counter()
    rtrom.march_batch(probs, steps)   # returns after the device finished
    t1 = time.perf_counter()
    prof = {}
    if profile:
        twin = [rtrom.Problem(s) for s in specs]
        if warmup > 0:
            rtrom.march_batch(twin, warmup)
        rtrom.profile_enable(True)
        rtrom.march_batch(twin, steps)
        prof = rtrom.profile_read()
        rtrom.profile_enable(False)
        for p in twin:
            p.close()
    return t1 - t0, probs, prof


def window_updates(probs, ca, first, steps):
    """Cell-angle SI updates, f-pass and SI bytes, and ROM update columns x
    cells of steps [first, first + steps) of every problem."""
    si_upd = 0
    rom_cell_cols = 0
    for p, c in zip(probs, ca):
        h = p.history()
        it = h["iters"][first:first + steps]
        si_upd += int(it.sum()) * c
        for key_u, key_r in (("ig_update", "rank_ig"), ("pc_update", "rank_pc")):
            upd, rank = h[key_u], h[key_r]
            for i in range(first, min(first + steps, len(upd))):
                if upd[i]:
                    r_old = int(rank[i - 1]) if i > 0 else 0
                    rom_cell_cols += (r_old + 1) * p.nc
    return si_upd, rom_cell_cols


def dg_half(s):
    """The instance in piecewise-linear DG form (Sec. 2.1 eq. DG, K = 1) on
    half its cells (every other cell's data, the same slab): as many
    unknowns as the finite-volume instance."""
    return s.replace(scheme="dg1", nx=(s.nx + 1) // 2, sigma_s=s.sigma_s[::2].copy(),
                     sigma_a=s.sigma_a[::2].copy(), source=s.source[::2].copy(),
                     f0=None if s.f0 is None else s.f0[::2].copy())


def bench_batch(rtrom, W, args, dg=False):
    specs = W.slab_batch()
    if dg:
        specs = [dg_half(s) for s in specs]
    cfg_steps = specs[0].nsteps
    steps = cfg_steps if args.steps is None else args.steps
    warm = 5 if args.warmup is None else args.warmup
    n = len(specs)
    res = {}
    for method in ("rom", "si_dsa"):
        ms = [s.replace(method=method) for s in specs]
        log(f"bench: batch512 {method} mixed: {warm} warmup + {steps} timed steps")
        t, probs, prof = timed_batch(rtrom, ms, warm, steps)
        ca = [p.nc * p.nv for p in probs]
        si_upd, rom_cc = window_updates(probs, ca, warm, steps)
        hist = [p.history() for p in probs]
        si_sw = sum(int(h["iters"][warm:warm + steps].sum()) for h in hist)
        res[method] = {"t": t, "prof": prof, "si_upd": si_upd, "rom_cc": rom_cc, "si_sw": si_sw,
                       "ca": sum(ca), "cells": sum(p.nc for p in probs),
                       "fp32": sum(p.stats()["fp32_sweeps"] for p in probs)}
        for p in probs:
            p.close()
    R, S = res["rom"], res["si_dsa"]
    value = n * steps / R["t"]
    si_val = n * steps / S["t"]
    fpass_bytes = steps * (FPASS_BYTES_PER_CELL_ANGLE * R["ca"] + FPASS_BYTES_PER_CELL * R["cells"])
    rom_bytes = ROM_BYTES_PER_CELL_COLUMN * R["rom_cc"]
    kernels = kernel_table(R["prof"], fpass_bytes, steps * SI_BYTES_PER_CELL * R["cells"], rom_bytes)
    # the roofline line reports the kernel that takes the longest in the timed
    # steps (every instance has at most 2048 cells: the wave-per-pair kernels)
    # among the SI launch and the f-pass.  The ROM post runs on the second
    # stream beside the f-pass: its event pair also brackets the wait for
    # compute units the f-pass holds, so its event time is not its duration
    # (rocprofv3: 222 us of kernel against ~315 us between its events), and
    # its kernel time is below the f-pass's
    dom = max(("slab_si", "slab_fpass"), key=lambda k: R["prof"].get(k, (0.0, 0))[0])
    if dom == "slab_si":
        roof = roofline_sweep(R["prof"], "slab_si", 1, R["si_upd"], "k_si_wave", SWEEP_FLOPS_DG1 if dg else None)
    else:
        roof = roofline_hbm(R["prof"], "slab_fpass", fpass_bytes, "k_fpass_dg" if dg else "k_fpass_wave")
    # the whole configured march of both methods, on fresh problems
    full = {}
    for method in ("rom", "si_dsa"):
        ms = [s.replace(method=method) for s in specs]
        log(f"bench: batch512 {method} mixed: full {cfg_steps}-step march")
        t, probs, _ = timed_batch(rtrom, ms, 0, cfg_steps, profile=False)
        hist = [p.history() for p in probs]
        sts = [p.stats() for p in probs]
        full[method] = {"instance_steps_per_s": n * cfg_steps / t, "ms_per_step": t / cfg_steps * 1e3,
                        "si_sweeps_per_step": sum(int(h["iters"].sum()) for h in hist) / (n * cfg_steps),
                        "fp32_sweeps_per_step": sum(st["fp32_sweeps"] for st in sts) / (n * cfg_steps),
                        "phase3_instances": sum(1 for st in sts if st["phase"] == 3),
                        "nonconverged_steps": sum(st["nonconverged_steps"] for st in sts)}
        for p in probs:
            p.close()
    full["speedup_vs_si_dsa"] = full["rom"]["instance_steps_per_s"] / full["si_dsa"]["instance_steps_per_s"]
    full["steps"] = cfg_steps
    # the same whole march with the variants of the method (every instance
    # has at most 2048 cells): the McClarren-Haut preconditioner alone and as
    # the hybrid with the ROM method (Sec. 3.3, 4.5), sequential correction
    # ROMs for iterations 1-2 (Sec. 3.2), BDF2 (Sec. 2.1) for both methods,
    # the FP64 mode of both methods, and the piecewise-linear DG scheme on
    # every instance (dg_half)
    variants = {}
    for name, method, kw in (("si_mh", "si_dsa", dict(precond="mh")), ("rom_mh_hybrid", "rom", dict(precond="mh")),
                             ("rom_levels2", "rom", dict(pc_levels=2)),
                             ("si_dsa_bdf2", "si_dsa", dict(time_scheme="bdf2")),
                             ("rom_bdf2", "rom", dict(time_scheme="bdf2")),
                             ("si_dsa_fp64", "si_dsa", dict(precision="fp64")), ("rom_fp64", "rom", dict(precision="fp64")),
                             ("si_dsa_dg1", "si_dsa", dict(scheme="dg1")), ("rom_dg1", "rom", dict(scheme="dg1"))):
        if args.no_variants or dg:
            break
        ms = [s.replace(method=method, **{k: v for k, v in kw.items() if k != "scheme"}) for s in specs]
        if kw.get("scheme") == "dg1":
            ms = [dg_half(s) for s in ms]
        log(f"bench: batch512 variant {name}: full {cfg_steps}-step march")
        t, probs, _ = timed_batch(rtrom, ms, 0, cfg_steps, profile=False)
        hist = [p.history() for p in probs]
        sts = [p.stats() for p in probs]
        variants[name] = {"instance_steps_per_s": n * cfg_steps / t, "ms_per_step": t / cfg_steps * 1e3,
                          "si_sweeps_per_step": sum(int(h["iters"].sum()) for h in hist) / (n * cfg_steps),
                          "nonconverged_steps": sum(st["nonconverged_steps"] for st in sts)}
        for p in probs:
            p.close()
    if variants:
        for a, b in (("rom_bdf2", "si_dsa_bdf2"), ("rom_fp64", "si_dsa_fp64"), ("rom_mh_hybrid", "si_mh"),
                     ("rom_dg1", "si_dsa_dg1")):
            variants[f"{a}_vs_{b}"] = variants[a]["instance_steps_per_s"] / variants[b]["instance_steps_per_s"]
    extra = {
        "si_dsa_instance_steps_per_s": si_val,
        "speedup_vs_si_dsa": value / si_val,
        "cell_angle_updates_per_s": (R["si_upd"] + 2 * steps * R["ca"]) / R["t"],
        "si_sweeps_per_step": R["si_sw"] / (n * steps),
        "si_dsa_si_sweeps_per_step": S["si_sw"] / (n * steps),
        "kernel_ms": kernel_ms(R["prof"]), "si_dsa_kernel_ms": kernel_ms(S["prof"]),
        "kernels": kernels,
        "full_march": full,
        "variants": variants,
    }
    config = {"workload": "batch512_slabs_dg1" if dg else "batch512_slabs", "instances": n, "steps": steps,
              "timed_steps": f"{warm + 1}..{warm + steps}",
              "cells": "64..1024 (DG-P1, two unknowns each)" if dg else "128..2048", "ordinates": "16/32/64",
              "dt": 0.01, "tol": 1e-8,
              "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refinement",
              "baseline_method": "si_dsa, same kernels and precision"}
    metric = "instance time steps/s (ROM-SI-DSA, 1e-8 rel tol)"
    cpu = None if args.no_cpu_baseline else cpu_baseline_batch(specs, min(steps, 20))
    return metric, "instance-steps/s", value, R["t"], steps, warm, config, roof, extra, cpu


def bench_single(rtrom, W, args):
    spec = W.slab_random_regions() if args.workload == "slab4096" else W.checkerboard()
    cfg_steps = spec.nsteps
    steps = cfg_steps if args.steps is None else args.steps
    warm = 5 if args.warmup is None else args.warmup
    nc, nv = spec.ncells, spec.nord
    res = {}
    for method in ("rom", "si_dsa"):
        log(f"bench: {args.workload} {method} mixed: {warm} warmup + {steps} timed steps")
        p = rtrom.Problem(spec.replace(method=method))
        if warm:
            p.march(warm)
        rtrom.profile_enable(True)
        t0 = time.perf_counter()
        p.march(steps)
        t1 = time.perf_counter()
        prof = rtrom.profile_read()
        rtrom.profile_enable(False)
        h = p.history()
        st = p.stats()
        res[method] = {"t": t1 - t0, "prof": prof, "si": int(h["iters"][warm:warm + steps].sum()), "st": st}
        p.close()
    full = {}
    for method in ("rom", "si_dsa"):
        log(f"bench: {args.workload} {method} mixed: full {cfg_steps}-step march")
        p = rtrom.Problem(spec.replace(method=method))
        t0 = time.perf_counter()
        p.march(cfg_steps)
        t = time.perf_counter() - t0
        st = p.stats()
        full[method] = {"steps_per_s": cfg_steps / t, "si_sweeps_per_step": st["si_iters_total"] / cfg_steps,
                        "fp32_sweeps_per_step": st["fp32_sweeps"] / cfg_steps, "n0": st["n0"], "n1": st["n1"]}
        p.close()
    full["speedup_vs_si_dsa"] = full["rom"]["steps_per_s"] / full["si_dsa"]["steps_per_s"]
    full["steps"] = cfg_steps
    # X-Y grid: the same whole march with the variants of the method
    # (McClarren-Haut alone and as the hybrid, Sec. 3.3 / 4.5; correction ROMs
    # for iterations 1-2, Sec. 3.2; BDF2, Sec. 2.1; the FP64 mode)
    variants = {}
    for name, method, kw in (("si_mh", "si_dsa", dict(precond="mh")), ("rom_mh_hybrid", "rom", dict(precond="mh")),
                             ("rom_levels2", "rom", dict(pc_levels=2)),
                             ("si_dsa_bdf2", "si_dsa", dict(time_scheme="bdf2")),
                             ("rom_bdf2", "rom", dict(time_scheme="bdf2")),
                             ("si_dsa_fp64", "si_dsa", dict(precision="fp64")), ("rom_fp64", "rom", dict(precision="fp64"))):
        if args.no_variants or spec.dim != 2:
            break
        log(f"bench: {args.workload} variant {name}: full {cfg_steps}-step march")
        p = rtrom.Problem(spec.replace(method=method, **kw))
        t0 = time.perf_counter()
        p.march(cfg_steps)
        t = time.perf_counter() - t0
        st = p.stats()
        variants[name] = {"steps_per_s": cfg_steps / t, "si_sweeps_per_step": st["si_iters_total"] / cfg_steps,
                          "nonconverged_steps": st["nonconverged_steps"]}
        p.close()
    if variants:
        for a, b in (("rom_bdf2", "si_dsa_bdf2"), ("rom_fp64", "si_dsa_fp64"), ("rom_mh_hybrid", "si_mh")):
            variants[f"{a}_vs_{b}"] = variants[a]["steps_per_s"] / variants[b]["steps_per_s"]
    R, S = res["rom"], res["si_dsa"]
    value = steps / R["t"]
    nfold = nv if spec.dim == 1 else nv // 2   # 2D sweeps the Omega_z > 0 half
    if spec.dim == 1:
        roof = roofline_sweep(R["prof"], "slab_si", 1, R["si"] * nc * nv, "k_si_slab")
    else:
        kinds = {k: v[0] for k, v in R["prof"].items() if v[1]}
        if max(kinds, key=kinds.get) == "plane_dsa":
            roof = roofline_dsa(R["prof"], nc, R["st"]["dsa_iters"])
        else:
            roof = roofline_sweep(R["prof"], "plane_sweep", 2, R["si"] * nc * nfold, "k_plane_sweep")
    extra = {
        "si_dsa_steps_per_s": steps / S["t"],
        "speedup_vs_si_dsa": S["t"] / R["t"],
        "cell_angle_updates_per_s": (R["si"] + 2 * steps) * nc * nv / R["t"],
        "si_sweeps_per_step": R["si"] / steps,
        "si_dsa_si_sweeps_per_step": S["si"] / steps,
        "kernel_ms": kernel_ms(R["prof"]), "si_dsa_kernel_ms": kernel_ms(S["prof"]),
        "full_march": full,
    }
    if variants:
        extra["variants"] = variants
    name = "slab4096_gl64_32regions" if spec.dim == 1 else "checkerboard256_cl16x8"
    config = {"workload": name, "cells": nc, "ordinates": nv, "dt": spec.dt, "steps": steps,
              "timed_steps": f"{warm + 1}..{warm + steps}", "tol": spec.tol, "method": "rom_si_dsa",
              "precision": "fp32 sweeps + fp64 refinement",
              "baseline_method": "si_dsa, same kernels and precision", "instances": 1}
    cpu = None if args.no_cpu_baseline else cpu_baseline_single(spec)
    return "time steps/s (ROM-SI-DSA, 1e-8 rel tol)", "steps/s", value, R["t"], steps, warm, config, roof, extra, cpu


# --------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample
# --------------------------------------------------------------------------

def cpu_baseline_single(spec, seconds_budget=20.0):
    """The FP64 oracle (same method) on the host, one core, the first steps of
    the same problem within a time budget."""
    import oracle
    model, ncpu = cpu_info()
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    n, t0 = 0, time.perf_counter()
    while n < spec.nsteps and time.perf_counter() - t0 < seconds_budget:
        o.step()
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {spec.nsteps} steps of the same problem, FP64 oracle, one thread",
            "host_cpu": model, "host_cpu_count": ncpu}


def _oracle_instance(args):
    spec, steps = args
    import oracle
    o = oracle.OracleProblem(spec.replace(precision="fp64"))
    o.march(steps)
    return steps


def cpu_baseline_batch(specs, steps):
    import multiprocessing as mp
    model, ncpu = cpu_info()
    cores = min(16, ncpu)
    sample = specs[: cores * 2]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        done = sum(pool.map(_oracle_instance, [(s, steps) for s in sample]))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "instance-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} of the {len(specs)} instances x their first {steps} steps, "
                      f"FP64 oracle, process pool of {cores}",
            "host_cpu": model, "host_cpu_count": ncpu}


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

def run_serving(rtrom, W, count, budget, slots, seed=5):
    """The serving stream: a closed-loop saturation run (everything submitted at once) gives the
    capacity; then Poisson arrivals at 80 % of it, with per-step and per-march
    latencies and the queueing delay seen by the client."""
    import numpy as np
    specs = W.serving_stream(seed=seed, count=count)
    srv = rtrom.Server(hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()
    tickets = [srv.submit(s) for s in specs]
    srv.drain()
    t_sat = time.perf_counter() - t0
    for t in tickets:
        srv.fetch(t)
    srv.close()
    log(f"bench: serving closed loop {t_sat:.2f} s")
    steps_total = sum(s.nsteps for s in specs)
    capacity = count / t_sat
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
    log(f"bench: serving open loop {t_open:.2f} s")
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


def bench_serving(rtrom, W, args):
    log(f"bench: serving stream of {args.requests} requests")
    res = run_serving(rtrom, W, args.requests, int(args.budget_gib * (1 << 30)), args.slots)
    config = {"workload": "serving_stream_grf_2d", "requests": args.requests,
              "grids": "64..512 squared", "ordinates": "32/64/128", "steps_each": "100..500",
              "method": "rom_si_dsa", "precision": "fp32 sweeps + fp64 refinement",
              "arrivals": "closed loop (value), then Poisson at 0.8 x capacity"}
    return ("instance time steps/s, serving (ROM-SI-DSA, 1e-8 rel tol)", "instance-steps/s",
            res["saturation_instance_steps_per_s"], res["saturation_s"], res["instance_steps"], 0, config, None,
            {"serving": res}, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the configured march)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps before them (default 5)")
    ap.add_argument("--workload", choices=("batch512", "batch512_dg", "slab4096", "checker256", "serving"),
                    default="batch512")
    ap.add_argument("--requests", type=int, default=24, help="serving: requests in the stream")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serving: HBM admission budget")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent problems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="batch512, checker256: skip the variant marches")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device five times (a plain copy of known size, "
                         "against which hardware byte counters are scaled)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every problem, and every instance of a batch, runs on one "
              "device; runs on several GPUs are not part of this library", file=sys.stderr)
        sys.exit(2)

    from paper_2603_19647_amd import rtrom
    from paper_2603_19647_amd import workloads as W

    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    if args.workload in ("batch512", "batch512_dg"):
        r = bench_batch(rtrom, W, args, dg=args.workload == "batch512_dg")
    elif args.workload == "serving":
        r = bench_serving(rtrom, W, args)
    else:
        r = bench_single(rtrom, W, args)
    metric, unit, value, t_timed, steps, warm, config, roof, extra, cpu = r
    if roof is not None:
        wl_name = {"slab4096_gl64_32regions": "slab4096", "checkerboard256_cl16x8": "checker256",
                   "batch512_slabs": "batch512", "batch512_slabs_dg1": "batch512_dg"}.get(config.get("workload"), "")
        roof["traffic"] = stored_traffic(roof["kernel"], wl_name)
    out = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": t_timed / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": config, "roofline": roof, "cpu_baseline": cpu, **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
