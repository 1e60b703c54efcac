#!/usr/bin/env python3
"""Benchmark of the parabolic sub-step on one MI355X.

Workload (a step = one parabolic step = temperature relaxation + 3 Picard
passes, each a coefficient build, a Gershgorin bound and one LIM pass of
2P-1 stencil sweeps): the 2D level-set case, 1024^2 periodic cells, two
phases with conductivities k0 (T/T0)^2, k0 = (1, 0.05), rho*C_v = (1, 5),
T lognormal (sigma 0.2), dt = 200x the explicit limit, 10 steps by
default.  Inputs are seeded and synthetic, resident in HBM before the timed
region.

Reported (one JSON line):
  value      FP64 cell-updates per second (N * sweeps / wall time of the steps)
  fp32       the same for the FP32 form and its speedup over FP64
  fp64_whole_step  FP64 with every step as one cooperative launch (P decided
             on the device) instead of one launch per block of stages
  roofline   dominant kernel (the blocked LIM sweep): algorithmic bytes per
             launch (N x 40 B x stages, an unfused sweep's compulsory bytes) /
             average launch time from HIP events on the library's stream;
             traffic = HBM bytes per launch from the committed rocprofv3
             FETCH_SIZE/WRITE_SIZE summary (null once the kernel changed)
  adjoint    adjoint / forward time on the 2048^2, 20-step adjoint workload
  bubbles3d  the 256^3 FP32 workload with the viscous part
  hyperbolic the hyperbolic part with pressure relaxation on the 1024^2
             shock-tube workload (one Godunov-HLLC sweep per axis per step):
             cell updates per second per sweep, and the sweep kernel's
             algorithmic bandwidth (9 doubles in, 9 out per cell and sweep)
  spitzer    FP64 on the same level-set fields with the Spitzer-Harm
             conductivity law (T^(5/2) over the Coulomb logarithm)
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell-update of one sweep launch: read v, rhs, Lambda,
# 1/C and write v, one word each (stencil neighbours come from cache).
BYTES_PER_UPDATE = {"fp64": 5 * 8, "fp32": 5 * 4}


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_tb2d_f64_levelset2d_1024.md")
SWEEP_SOURCES = ("tlim_sweep.hip", "tlim_device.h")


def sweep_source_digest():
    """Digest of the sources that define the blocked sweep kernel."""
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_00282_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic():
    """HBM bytes per launch of the FP64 blocked sweep from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (each scaled by what the same
    counter reads for a plain copy of known size).  None when the summary is
    missing or the kernel's sources changed since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines() if ": " in line and " " not in
                      line.split(": ", 1)[0])
    except OSError:
        return None
    if kv.get("source_digest", "").strip() != sweep_source_digest():
        return None
    try:
        return float(kv["sweep_fp64_traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_steps(solver, wl, opts, steps, reset=True):
    import torch
    if reset:
        solver.set_workload(wl)
    oc = opts.c()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = solver.advance_raw(oc)
        if st != 0:
            raise RuntimeError(f"tlim_advance returned {st}")
    st = solver.finish()  # the last step's readback is checked inside the timed region
    if st != 0:
        raise RuntimeError(f"tlim_finish returned {st}")
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def measure(precision, wl, tau, steps, warmup, whole=0):
    """Wall time of `steps` steps from the initial state on a fresh context
    (no schedule history), after `warmup` steps on another context; then an
    identical untimed run with sweep events for the sweep count and the
    per-launch kernel time."""
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    opts = StepOpts(dt=tau, passes=wl["passes"], whole_step=whole)
    if warmup:
        w = Solver(wl["n"], wl["h"], wl["bc"], precision=precision)
        run_steps(w, wl, opts, warmup)
        del w
    s = Solver(wl["n"], wl["h"], wl["bc"], precision=precision)
    s.set_workload(wl)
    wall = run_steps(s, wl, opts, steps, reset=False)
    s2 = Solver(wl["n"], wl["h"], wl["bc"], precision=precision)
    s2.set_workload(wl)
    sweeps = launches = 0
    sweep_ms = 0.0
    predicted = mispredicted = 0
    # the blocked-sweep launches alone (a step run as one cooperative launch
    # of the whole-step kernel is left out of these): the roofline's kernel
    tb_sweeps = tb_launches = 0
    tb_ms = 0.0
    topts = StepOpts(dt=tau, passes=wl["passes"], time_sweeps=1, whole_step=whole)
    for _ in range(steps):
        st, rep = s2.advance(topts)
        sweeps += rep["sweeps"]
        launches += rep["sweep_launches"]
        sweep_ms += rep["sweep_ms"]
        predicted += rep["predicted"]
        mispredicted += rep["mispredicted"]
        if rep["sweep_launches"] > 1:
            tb_sweeps += rep["sweeps"]
            tb_launches += rep["sweep_launches"]
            tb_ms += rep["sweep_ms"]
    N = s.N
    return dict(wall_s=wall, sweeps=sweeps, launches=launches, sweep_ms=sweep_ms, N=N,
                gupd=N * sweeps / wall / 1e9, predicted_steps=predicted, mispredicted_steps=mispredicted,
                tb_sweeps=tb_sweeps, tb_launches=tb_launches, tb_ms=tb_ms)


def adjoint_ratio():
    """Adjoint / forward time on the 2048^2 level-set workload, 20 steps,
    FP64, checkpoint every step (forward includes writing the checkpoints)."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    wl = W.levelset2d_adjoint(2048, 20)
    s = Solver(wl["n"], wl["h"], wl["bc"])
    s.set_workload(wl)
    tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
    opts = StepOpts(dt=tau, passes=3)
    steps = wl["steps"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    TN = s.get_field("T1")
    g = TN - torch.from_numpy(wl["fields"]["T1"]).to(TN.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adjoint(opts, steps, 1, ckpt, lam, g)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    return dict(workload="levelset2d_adjoint 2048^2, 20 steps x 3 passes, FP64, checkpoint every step",
                forward_s=round(t_fwd, 4), adjoint_s=round(t_adj, 4), ratio=round(t_adj / t_fwd, 3))


def bubbles3d_rate(n=256, steps=5):
    """The 3D bubbles workload (256^3 periodic, FP32 sweeps, viscous part on,
    5 steps): whole-step throughput and sweep-kernel rate."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    wl = W.bubbles3d(n, steps=steps)
    s = Solver(wl["n"], wl["h"], wl["bc"], precision="fp32")
    s.set_workload(wl)
    tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
    opts = StepOpts(dt=tau, passes=wl["passes"], do_viscous=1)
    run_steps(s, wl, opts, 1)  # warm-up step on the same fields, then start over
    s.set_workload(wl)
    # timed: the steps with reports (the viscous part reads its bounds back anyway)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps = 0
    for _ in range(steps):
        st, rep = s.advance(opts)
        if st != 0:
            raise RuntimeError(f"tlim_advance returned {st}")
        sweeps += rep["sweeps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(workload=f"bubbles3d {n}^3 periodic, FP32 sweeps, viscous part, {steps} steps",
                value=round(s.N * sweeps / wall / 1e9, 3), unit="Gcell-updates/s",
                ms_per_step=round(wall / steps * 1e3, 3), sweeps=sweeps)


def hyperbolic_rate(n=1024, steps=10, warmup=2):
    """Whole-step throughput of the hyperbolic part: `steps` steps at the
    CFL-0.4 time step of the initial state, inputs resident on the device."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver
    wl = W.shocktube2d(n, steps=steps)
    s = Solver(wl["n"], wl["h"], wl["bc"])
    s.set_workload(wl)
    dt = s.hyperbolic_dt(wl["cfl"])
    for _ in range(warmup):
        s.advance_hyperbolic(dt, report=False)
    s.set_workload(wl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.advance_hyperbolic(dt, report=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st, bad = s.advance_hyperbolic(dt)  # the state is still admissible
    if st != 0 or bad:
        raise RuntimeError(f"hyperbolic step failed: status {st}, {bad} bad cells")
    N = s.N
    sweeps = 2 * steps
    return dict(workload=f"shocktube2d {n}^2 periodic, two SG phases, Godunov-HLLC + pressure relaxation, "
                         f"{steps} steps at CFL 0.4",
                value=round(N * sweeps / wall / 1e9, 3), unit="Gcell-updates/s (per directional sweep)",
                ms_per_step=round(wall / steps * 1e3, 4),
                algorithmic_GBs=round(N * 144 * sweeps / wall / 1e9, 1))


def cpu_baseline(wl, tau, budget_s=12.0):
    """The FP64 oracle, as it is, on whole steps of the same workload until
    about budget_s of CPU time has passed."""
    from oracle import oracle as orc
    orc.build(force=False)
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    f = {k: v.copy() for k, v in wl["fields"].items()}
    opts = orc.StepOpts(tau=tau, passes=wl["passes"])
    updates, steps = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < wl["steps"]:
        st, rep = orc.step(g, wl["phases"], opts, f)
        updates += wl["n"][0] * wl["n"][1] * wl["n"][2] * sum(2 * p - 1 for p in rep["P"])
        steps += 1
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=round(updates / dt / 1e9, 5), unit="Gcell-updates/s", cores=cores, kind="oracle",
                sample=f"first {steps} of the {wl['steps']} steps of the benchmark workload "
                       f"({wl['n'][0]}x{wl['n'][1]}), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="cells per axis of the level-set workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-spitzer", action="store_true")
    ap.add_argument("--no-hyperbolic", action="store_true")
    ap.add_argument("--hyperbolic-only", action="store_true",
                    help="run only the hyperbolic measurement and print its JSON (for profiling that path)")
    ap.add_argument("--workload", choices=("levelset2d", "levelset2d_spitzer"), default="levelset2d",
                    help="main workload (levelset2d_spitzer: the same fields with the Spitzer-Harm law, "
                         "for profiling that path)")
    ap.add_argument("--no-whole", action="store_true",
                    help="never run a step as one cooperative launch (also not the first step): for profilers")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see the sharding "
              "notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver

    if args.hyperbolic_only:
        print(json.dumps(hyperbolic_rate(n=args.n, steps=args.steps, warmup=args.warmup)), flush=True)
        return

    wl = getattr(W, args.workload)(args.n, steps=args.steps)
    probe = Solver(wl["n"], wl["h"], wl["bc"])
    probe.set_workload(wl)
    lam = probe.spectral_bound()
    tau = wl["dt_factor"] * 2.0 / lam
    del probe
    log(f"workload {args.workload} {args.n}^2, tau*lambda_G = {tau * lam:.1f}")

    whole = 2 if args.no_whole else 0
    r64 = measure("fp64", wl, tau, args.steps, args.warmup, whole=whole)
    log("fp64", r64)
    r32 = None if args.fp64_only else measure("fp32", wl, tau, args.steps, args.warmup, whole=whole)
    if r32:
        log("fp32", r32)
    rw = None if args.fp64_only or args.no_whole else measure("fp64", wl, tau, args.steps, args.warmup, whole=1)
    if rw:
        log("fp64 whole-step", rw)
    adj = None if args.no_adjoint else adjoint_ratio()
    if adj:
        log("adjoint", adj)
    b3 = None if args.no_3d or args.fp64_only else bubbles3d_rate()
    if b3:
        log("bubbles3d", b3)
    hy = None if args.no_hyperbolic or args.fp64_only or args.workload != "levelset2d" else hyperbolic_rate()
    if hy:
        log("hyperbolic", hy)
    sh = None
    if not (args.no_spitzer or args.fp64_only or args.workload != "levelset2d"):
        wls = W.levelset2d_spitzer(args.n, steps=args.steps)
        probe = Solver(wls["n"], wls["h"], wls["bc"])
        probe.set_workload(wls)
        lam_s = probe.spectral_bound()
        del probe
        tau_s = wls["dt_factor"] * 2.0 / lam_s
        rs = measure("fp64", wls, tau_s, args.steps, args.warmup, whole=whole)
        log("spitzer fp64", rs)
        sh = {"workload": f"levelset2d_spitzer {args.n}^2, Spitzer-Harm law (n = 5/2, Coulomb logarithm), "
                          f"FP64, 200x, 3 passes, {args.steps} steps",
              "value": round(rs["gupd"], 4), "unit": "Gcell-updates/s",
              "ms_per_step": round(rs["wall_s"] / args.steps * 1e3, 4), "sweeps": rs["sweeps"],
              "tau_lambda_G": round(tau_s * lam_s, 1)}

    avg_launch_ms = r64["tb_ms"] / max(r64["tb_launches"], 1)
    bytes_per_launch = r64["N"] * BYTES_PER_UPDATE["fp64"] * (r64["tb_sweeps"] / max(r64["tb_launches"], 1))
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if avg_launch_ms > 0 else None
    traffic = pmc_traffic() if args.n == 1024 and args.workload == "levelset2d" else None
    dram_gbs = traffic / (avg_launch_ms * 1e-3) / 1e9 if traffic and avg_launch_ms > 0 else None
    out = {
        "metric": "Gcell-updates/s per Chebyshev sweep (FP64 vs FP32), HBM GB/s, adjoint/fwd",
        "value": round(r64["gupd"], 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["wall_s"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"levelset2d {args.n}x{args.n} periodic, two phases, k=k0 (T/T0)^2, "
                               f"dt=200x explicit limit, 3 Picard passes, {args.steps} steps"
                   if args.workload == "levelset2d" else
                   f"levelset2d_spitzer {args.n}x{args.n} periodic, two phases, Spitzer-Harm law, "
                   f"dt=200x explicit limit, 3 Picard passes, {args.steps} steps",
                   "cells": r64["N"], "sweeps_per_run": r64["sweeps"],
                   "predicted_steps": r64["predicted_steps"], "mispredicted_steps": r64["mispredicted_steps"]},
        "sweep_kernel_gupd": round(r64["N"] * r64["sweeps"] / (r64["sweep_ms"] * 1e-3) / 1e9, 2)
        if r64["sweep_ms"] > 0 else None,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": int(traffic) if traffic else None,
                     "kernel": "LIM sweep (FP64, blocked)", "avg_launch_us": round(avg_launch_ms * 1e3, 3),
                     "bytes_per_launch": int(bytes_per_launch),
                     "dram_GBs": round(dram_gbs, 1) if dram_gbs else None,
                     "dram_frac": round(dram_gbs / HBM_PEAK_GBS, 4) if dram_gbs else None},
    }
    if r32:
        l32 = r32["sweep_ms"] / max(r32["launches"], 1)
        b32 = r32["N"] * BYTES_PER_UPDATE["fp32"] * (r32["sweeps"] / max(r32["launches"], 1))
        out["fp32"] = {"value": round(r32["gupd"], 4), "unit": "Gcell-updates/s",
                       "speedup_vs_fp64": round(r32["gupd"] / r64["gupd"], 3),
                       "ms_per_step": round(r32["wall_s"] / args.steps * 1e3, 4),
                       "sweep_GBs": round(b32 / (l32 * 1e-3) / 1e9, 1) if l32 > 0 else None}
    if rw:
        out["fp64_whole_step"] = {"value": round(rw["gupd"], 4), "unit": "Gcell-updates/s",
                                  "ms_per_step": round(rw["wall_s"] / args.steps * 1e3, 4),
                                  "launches_per_step": rw["launches"] / args.steps}
    if adj:
        out["adjoint"] = adj
    if b3:
        out["bubbles3d"] = b3
    if sh:
        out["spitzer"] = sh
    if hy:
        out["hyperbolic"] = hy
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, tau)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
