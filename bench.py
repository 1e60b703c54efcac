#!/usr/bin/env python3
"""Benchmark of the parabolic sub-step on one MI355X.

Headline workload (a step = one parabolic step = temperature relaxation + 3
Picard passes, each a coefficient build, a Gershgorin bound and one LIM pass
of 2P-1 stencil sweeps): the 2D level-set case, 1024^2 periodic cells, two
phases with conductivities k0 (T/T0)^2, k0 = (1, 0.05), rho*C_v = (1, 5),
T lognormal (sigma 0.2), dt = 200x the explicit limit, 10 steps by
default.  Inputs are seeded and synthetic, resident in HBM before the timed
region.

Reported (one JSON line):
  value      FP64 cell-updates per second: N * sweeps / wall time of the
             steps (timed region bracketed by device synchronisation)
  roofline   the dominant kernel, the blocked FP64 LIM sweep: a launch runs
             K stages on tiles held on chip, so its compulsory HBM traffic
             is one read of v, g, Lambda, 1/C and one write of v per cell
             (5 words = 40 B per cell per launch, whatever K is);
             achieved = N x 40 B / average launch time (HIP events on the
             library's stream), against the 8 TB/s HBM peak.  Beside it:
             traffic = HBM bytes per launch from the committed rocprofv3
             FETCH_SIZE / WRITE_SIZE summary (null once the kernel changed),
             its ratio to the compulsory bytes, the FP64 VALU fraction, the
             unfused-equivalent bandwidth (K x 40 B per cell) and a plain
             1 GiB device copy timed here (the measured copy peak)
  fp32       the FP32 form: rate, speedup over FP64, the same roofline for
             its blocked kernel (5 x 4 B per cell per launch), and the
             per-field error against the FP64 oracle
  fp64_whole_step  FP64 with every step as one cooperative launch
  adjoint    adjoint / forward time on the 2048^2, 20-step adjoint workload
  bubbles3d  the 256^3 FP32 workload with the viscous part (5 steps)
  interface3d  the 512^3 FP32 workload (x adiabatic, contrast 100): forward
             rate over 10 steps and adjoint / forward with checkpoints every
             2 steps
  hyperbolic the hyperbolic part with pressure relaxation on the 1024^2
             shock-tube workload
  spitzer    FP64 on the level-set fields with the Spitzer-Harm law
  cpu_baseline  the FP64 oracle on a bounded sample of the headline
             workload, with all host threads and with one
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
FP64_VALU_PEAK_TFLOPS = 78.6
FP32_VALU_PEAK_TFLOPS = 157.3
# Compulsory bytes of one blocked launch per cell: read v, g, Lambda, 1/C and
# write v once, one word each.
WORDS_PER_CELL_LAUNCH = 5
WORD = {"fp64": 8, "fp32": 4}
# Floating-point operations of one stage per cell: the four face terms
# kappa_f (v - v_f) (4 subtractions, 1 product, 3 fused multiply-adds) and
# c_m (g + tau b v - S) (1 fused multiply-add, 1 subtraction, 1 product),
# counting a fused multiply-add as 2.
FLOPS_PER_CELL_STAGE = 15

PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_tb2d_levelset2d_1024.md")
SWEEP_SOURCES = ("tlim_sweep.hip", "tlim_device.h", "tlim_sweep.h")


def sweep_source_digest():
    """Digest of the sources that define the blocked sweep kernel."""
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_00282_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(prec):
    """L2-to-memory bytes per launch of the blocked sweep of precision `prec`
    from the committed rocprofv3 summary of the raw request counters
    (checked on a plain 1 GiB copy).  None when the summary is missing or
    the kernel's sources changed since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as fh:
            kv = dict(line.split(": ", 1) for line in fh.read().splitlines()
                      if ": " in line and " " not in line.split(": ", 1)[0])
    except OSError:
        return None
    if kv.get("source_digest", "").strip() != sweep_source_digest():
        return None
    try:
        return float(kv[f"sweep_{prec}_traffic_bytes_per_launch"])
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
            raise RuntimeError(f"tlim_advance_parabolic returned {st}")
    st = solver.finish()  # the last step's readback is checked inside the timed region
    if st != 0:
        raise RuntimeError(f"tlim_finish returned {st}")
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def measure(precision, wl, tau, steps, warmup, whole=0):
    """Wall time of `steps` steps from the initial state on a fresh context
    (no schedule history), after `warmup` steps on another context; then an
    identical untimed run with sweep events for the sweep count and the
    per-launch kernel time.  Returns the numbers and the final T1 and
    alpha2 of the timed run (host arrays)."""
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    opts = StepOpts(dt=tau, passes=wl["passes"], whole_step=whole)
    if warmup:
        with Solver(wl["n"], wl["h"], wl["bc"], precision=precision) as w:
            run_steps(w, wl, opts, warmup)
    with Solver(wl["n"], wl["h"], wl["bc"], precision=precision) as s:
        s.set_workload(wl)
        wall = run_steps(s, wl, opts, steps, reset=False)
        final = {k: s.get_field(k).cpu().numpy() for k in ("T1", "alpha2")}
        N = s.N
    sweeps = launches = 0
    sweep_ms = 0.0
    predicted = mispredicted = 0
    # the blocked-sweep launches that the library times (the roofline's
    # kernel): those of the passes enqueued behind earlier device work of
    # their step, in the steps with a predicted schedule (a whole-step launch
    # and a pass enqueued right after a readback are not timed)
    tb_sweeps = tb_launches = 0
    tb_ms = 0.0
    topts = StepOpts(dt=tau, passes=wl["passes"], time_sweeps=1, whole_step=whole)
    with Solver(wl["n"], wl["h"], wl["bc"], precision=precision) as s2:
        s2.set_workload(wl)
        for _ in range(steps):
            st, rep = s2.advance(topts)
            sweeps += rep["sweeps"]
            launches += rep["sweep_launches"]
            sweep_ms += rep["sweep_ms"]
            predicted += rep["predicted"]
            mispredicted += rep["mispredicted"]
            if rep["predicted"]:
                tb_sweeps += rep["timed_sweeps"]
                tb_launches += rep["timed_launches"]
                tb_ms += rep["sweep_ms"]
    return dict(wall_s=wall, sweeps=sweeps, launches=launches, sweep_ms=sweep_ms, N=N,
                gupd=N * sweeps / wall / 1e9, predicted_steps=predicted, mispredicted_steps=mispredicted,
                tb_sweeps=tb_sweeps, tb_launches=tb_launches, tb_ms=tb_ms, final=final)


def roofline(r, prec, copy_peak):
    """Roofline figures of the blocked sweep from a measure() result."""
    if not r["tb_launches"] or r["tb_ms"] <= 0:
        return None
    N = r["N"]
    avg_s = r["tb_ms"] * 1e-3 / r["tb_launches"]
    stages = r["tb_sweeps"] / r["tb_launches"]
    compulsory = N * WORDS_PER_CELL_LAUNCH * WORD[prec]
    achieved = compulsory / avg_s / 1e9
    traffic = pmc_traffic(prec) if N == 1 << 20 else None
    flops = N * stages * FLOPS_PER_CELL_STAGE / avg_s / 1e12
    peak_alu = FP64_VALU_PEAK_TFLOPS if prec == "fp64" else FP32_VALU_PEAK_TFLOPS
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": int(traffic) if traffic else None,
           "kernel": ("k_tb2d<double, 16, 1> (blocked LIM stages, 64 x 128 tiles)" if prec == "fp64" else
                      "k_tb2d<float, 16, 2> (blocked LIM stages, 128 x 64 tiles, two cells per lane)"),
           "avg_launch_us": round(avg_s * 1e6, 3), "stages_per_launch": round(stages, 3),
           "compulsory_bytes_per_launch": int(compulsory),
           "traffic_over_compulsory": round(traffic / compulsory, 3) if traffic else None,
           "dram_GBs": round(traffic / avg_s / 1e9, 1) if traffic else None,
           "effective_unfused_GBs": round(achieved * stages, 1),
           "valu": {"flops_per_cell_stage": FLOPS_PER_CELL_STAGE, "achieved_TFLOPs": round(flops, 3),
                    "peak_TFLOPs": peak_alu, "frac": round(flops / peak_alu, 4)}}
    if copy_peak:
        out["copy_peak_GBs"] = copy_peak
        out["frac_of_copy_peak"] = round(achieved / copy_peak, 4)
    return out


def copy_peak(gib=1.0, reps=10):
    """Bandwidth of a plain device-to-device copy of `gib` GiB of float64
    (read + write bytes over the average time of `reps` copies)."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)


def adjoint_ratio():
    """Adjoint / forward time on the 2048^2 level-set workload, 20 steps,
    FP64, checkpoint every step (forward includes writing the checkpoints)."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    wl = W.levelset2d_adjoint(2048, 20)
    with Solver(wl["n"], wl["h"], wl["bc"]) as s:
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
    5 steps): whole-step throughput."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    wl = W.bubbles3d(n, steps=steps)
    with Solver(wl["n"], wl["h"], wl["bc"], precision="fp32") as s:
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
                raise RuntimeError(f"tlim_advance_parabolic returned {st}")
            sweeps += rep["sweeps"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        N = s.N
    return dict(workload=f"bubbles3d {n}^3 periodic, FP32 sweeps, viscous part, {steps} steps",
                value=round(N * sweeps / wall / 1e9, 3), unit="Gcell-updates/s",
                ms_per_step=round(wall / steps * 1e3, 3), sweeps=sweeps)


def adjoint_pair(wl, precision, steps, ckpt_every):
    """Checkpointed forward and adjoint of `steps` steps of workload wl in a
    context of `precision`, timed each (seconds)."""
    import torch
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    with Solver(wl["n"], wl["h"], wl["bc"], precision=precision) as s:
        s.set_workload(wl)
        tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
        opts = StepOpts(dt=tau, passes=wl["passes"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ckpt, lam = s.forward_checkpointed(opts, steps, ckpt_every)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        TN = s.get_field("T1")
        g = TN - torch.from_numpy(wl["fields"]["T1"]).to(TN.device)
        del TN
        # the workspace is allocated once per solver and reused by every
        # adjoint call: outside the timed region (one allocation above about
        # 110 GiB takes seconds on this allocator)
        s.adjoint_workspace(opts, steps, ckpt_every, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.adjoint(opts, steps, ckpt_every, ckpt, lam, g)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        del ckpt, g
    torch.cuda.empty_cache()
    return t_fwd, t_adj


def interface3d_rate(n=512, steps=10, ckpt_every=2):
    """The 3D interface workload (512^3, x adiabatic, contrast 100) in an FP32
    context: forward throughput over `steps` steps, then the checkpointed
    forward (every `ckpt_every` steps) and the adjoint, timed each; and the
    same pair in an FP64 context."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    wl = W.interface3d(n, steps=steps)
    log(f"interface3d {n}^3 generated")
    with Solver(wl["n"], wl["h"], wl["bc"], precision="fp32") as s:
        s.set_workload(wl)
        tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
        opts = StepOpts(dt=tau, passes=wl["passes"])
        run_steps(s, wl, opts, 1)  # warm-up step, then start over
        s.set_workload(wl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps = 0
        for _ in range(steps):
            st, rep = s.advance(opts)
            if st != 0:
                raise RuntimeError(f"tlim_advance_parabolic returned {st}")
            sweeps += rep["sweeps"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        log(f"interface3d forward {wall:.3f} s")
        N = s.N
    torch.cuda.empty_cache()
    t_fwd, t_adj = adjoint_pair(wl, "fp32", steps, ckpt_every)
    log(f"interface3d FP32 context: checkpointed forward {t_fwd:.3f} s, adjoint {t_adj:.3f} s")
    f64_fwd, f64_adj = adjoint_pair(wl, "fp64", steps, ckpt_every)
    log(f"interface3d FP64 context: checkpointed forward {f64_fwd:.3f} s, adjoint {f64_adj:.3f} s")
    return dict(workload=f"interface3d {n}^3, x adiabatic, k0 = (1, 0.01), FP32 sweeps with FP64 state, "
                         f"sums and relaxation, {steps} steps x 3 passes",
                value=round(N * sweeps / wall / 1e9, 3), unit="Gcell-updates/s",
                ms_per_step=round(wall / steps * 1e3, 3), sweeps=sweeps,
                adjoint={"checkpoint_every": ckpt_every, "forward_checkpointed_s": round(t_fwd, 4),
                         "adjoint_s": round(t_adj, 4), "ratio": round(t_adj / t_fwd, 3),
                         "note": "the adjoint recomputes each step from its checkpoint and reverses it in FP64",
                         "fp64_context": {"forward_checkpointed_s": round(f64_fwd, 4), "adjoint_s": round(f64_adj, 4),
                                          "ratio": round(f64_adj / f64_fwd, 3)}})


def hyperbolic_rate(n=1024, steps=10, warmup=2):
    """Whole-step throughput of the hyperbolic part: `steps` steps at the
    CFL-0.4 time step of the initial state, inputs resident on the device."""
    import torch
    from paper_2106_00282_amd import workloads as W
    from paper_2106_00282_amd.tlim import Solver
    wl = W.shocktube2d(n, steps=steps)
    with Solver(wl["n"], wl["h"], wl["bc"]) as s:
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle (its libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(wl, tau, budget_s=12.0):
    """The FP64 oracle, as it is, on whole steps of the same workload: with
    every host thread until about budget_s has passed, then one step on one
    thread.  Returns the figures and the oracle's state and schedule after
    the multi-threaded steps."""
    from oracle import oracle as orc
    orc.build(force=False)
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    N = wl["n"][0] * wl["n"][1] * wl["n"][2]
    opts = orc.StepOpts(tau=tau, passes=wl["passes"])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    _omp_threads(threads)
    f = {k: v.copy() for k, v in wl["fields"].items()}
    updates, steps, lams = 0, 0, []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < wl["steps"]:
        st, rep = orc.step(g, wl["phases"], opts, f)
        updates += N * sum(2 * p - 1 for p in rep["P"])
        lams.append(rep["lambda_G"])
        steps += 1
    dt = time.perf_counter() - t0
    one = None
    if _omp_threads(1):
        f1 = {k: v.copy() for k, v in wl["fields"].items()}
        t1 = time.perf_counter()
        st, rep = orc.step(g, wl["phases"], opts, f1)
        d1 = time.perf_counter() - t1
        one = {"value": round(N * sum(2 * p - 1 for p in rep["P"]) / d1 / 1e9, 5), "unit": "Gcell-updates/s",
               "threads": 1, "sample": f"first step of the benchmark workload, {d1:.1f} s"}
        _omp_threads(threads)
    out = dict(value=round(updates / dt / 1e9, 5), unit="Gcell-updates/s", cores=threads, kind="oracle",
               sample=f"first {steps} of the {wl['steps']} steps of the benchmark workload "
                      f"({wl['n'][0]}x{wl['n'][1]}), {dt:.1f} s",
               cpu_model=cpu_model(), host_cpus=os.cpu_count())
    if one:
        out["single_thread"] = one
    return out, f, lams


def field_errors_vs_oracle(wl, tau, f_orc, lams, precision):
    """The GPU path of `precision` for the oracle's steps with the oracle's
    schedule frozen in: max-norm relative error per field."""
    import numpy as np
    from paper_2106_00282_amd.tlim import Solver, StepOpts
    with Solver(wl["n"], wl["h"], wl["bc"], precision=precision) as s:
        s.set_workload(wl)
        for lam in lams:
            st, _ = s.advance(StepOpts(dt=tau, passes=wl["passes"], frozen_lambda=lam))
            if st != 0:
                raise RuntimeError(f"tlim_advance_parabolic returned {st}")
        out = {}
        for k in ("T1", "T2", "alpha2"):
            a = s.get_field(k).cpu().numpy()
            out[k] = float(np.abs(a - f_orc[k]).max() / np.abs(f_orc[k]).max())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="cells per axis of the level-set workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip both 3D workloads")
    ap.add_argument("--no-c5", action="store_true", help="skip the 512^3 interface workload")
    ap.add_argument("--c5-n", type=int, default=512)
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-spitzer", action="store_true")
    ap.add_argument("--no-hyperbolic", action="store_true")
    ap.add_argument("--hyperbolic-only", action="store_true",
                    help="run only the hyperbolic measurement and print its JSON (for profiling that path)")
    ap.add_argument("--copy-only", action="store_true",
                    help="run only the 1 GiB copy and print its bandwidth (counter calibration)")
    ap.add_argument("--c3-only", action="store_true",
                    help="run only the 256^3 bubbles measurement and print its JSON (for profiling)")
    ap.add_argument("--c5-only", action="store_true",
                    help="run only the 512^3 interface measurement and print its JSON (for profiling)")
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
    if args.copy_only:
        print(json.dumps({"copy_peak_GBs": copy_peak()}), flush=True)
        return
    if args.c3_only:
        print(json.dumps(bubbles3d_rate(steps=args.steps)), flush=True)
        return
    if args.c5_only:
        print(json.dumps(interface3d_rate(n=args.c5_n, steps=args.steps)), flush=True)
        return

    wl = getattr(W, args.workload)(args.n, steps=args.steps)
    with Solver(wl["n"], wl["h"], wl["bc"]) as probe:
        probe.set_workload(wl)
        lam = probe.spectral_bound()
    tau = wl["dt_factor"] * 2.0 / lam
    log(f"workload {args.workload} {args.n}^2, tau*lambda_G = {tau * lam:.1f}")

    cp = None if args.no_copy else copy_peak()
    log(f"copy peak (1 GiB float64 device copy): {cp} GB/s")
    whole = 2 if args.no_whole else 0
    r64 = measure("fp64", wl, tau, args.steps, args.warmup, whole=whole)
    log("fp64", {k: v for k, v in r64.items() if k != "final"})
    r32 = None if args.fp64_only or args.no_fp32 else measure("fp32", wl, tau, args.steps, args.warmup, whole=whole)
    if r32:
        log("fp32", {k: v for k, v in r32.items() if k != "final"})
    rw = None if args.fp64_only or args.no_whole else measure("fp64", wl, tau, args.steps, args.warmup, whole=1)
    if rw:
        log("fp64 whole-step", {k: v for k, v in rw.items() if k != "final"})
    adj = None if args.no_adjoint or args.fp64_only else adjoint_ratio()
    if adj:
        log("adjoint", adj)
    b3 = None if args.no_3d or args.fp64_only else bubbles3d_rate()
    if b3:
        log("bubbles3d", b3)
    c5 = None if args.no_3d or args.no_c5 or args.fp64_only else interface3d_rate(n=args.c5_n, steps=10)
    if c5:
        log("interface3d", c5)
    hy = None if args.no_hyperbolic or args.fp64_only or args.workload != "levelset2d" else hyperbolic_rate()
    if hy:
        log("hyperbolic", hy)
    sh = None
    if not (args.no_spitzer or args.fp64_only or args.workload != "levelset2d"):
        wls = W.levelset2d_spitzer(args.n, steps=args.steps)
        with Solver(wls["n"], wls["h"], wls["bc"]) as probe:
            probe.set_workload(wls)
            lam_s = probe.spectral_bound()
        tau_s = wls["dt_factor"] * 2.0 / lam_s
        rs = measure("fp64", wls, tau_s, args.steps, args.warmup, whole=whole)
        log("spitzer fp64", {k: v for k, v in rs.items() if k != "final"})
        sh = {"workload": f"levelset2d_spitzer {args.n}^2, Spitzer-Harm law (n = 5/2, Coulomb logarithm), "
                          f"FP64, 200x, 3 passes, {args.steps} steps",
              "value": round(rs["gupd"], 4), "unit": "Gcell-updates/s",
              "ms_per_step": round(rs["wall_s"] / args.steps * 1e3, 4), "sweeps": rs["sweeps"],
              "tau_lambda_G": round(tau_s * lam_s, 1)}

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
        "sweep_kernel_gupd": round(r64["N"] * r64["tb_sweeps"] / (r64["tb_ms"] * 1e-3) / 1e9, 2)
        if r64["tb_ms"] > 0 else None,
        "roofline": roofline(r64, "fp64", cp),
    }
    if r32:
        import numpy as np
        out["fp32"] = {"value": round(r32["gupd"], 4), "unit": "Gcell-updates/s",
                       "speedup_vs_fp64": round(r32["gupd"] / r64["gupd"], 3),
                       "ms_per_step": round(r32["wall_s"] / args.steps * 1e3, 4),
                       "roofline": roofline(r32, "fp32", cp),
                       "err_vs_fp64_path": {k: float(np.abs(r32["final"][k] - r64["final"][k]).max()
                                                     / np.abs(r64["final"][k]).max())
                                            for k in ("T1", "alpha2")}}
    if rw:
        out["fp64_whole_step"] = {"value": round(rw["gupd"], 4), "unit": "Gcell-updates/s",
                                  "ms_per_step": round(rw["wall_s"] / args.steps * 1e3, 4),
                                  "launches_per_step": rw["launches"] / args.steps}
    if adj:
        out["adjoint"] = adj
    if b3:
        out["bubbles3d"] = b3
    if c5:
        out["interface3d"] = c5
    if sh:
        out["spitzer"] = sh
    if hy:
        out["hyperbolic"] = hy
    if not args.no_cpu:
        cb, f_orc, lams = cpu_baseline(wl, tau)
        log("cpu_baseline", cb)
        out["cpu_baseline"] = cb
        # per-field error of both precisions against the FP64 oracle over the
        # steps the baseline ran (the oracle's schedule frozen into the GPU runs)
        errs = {"steps": len(lams), "fp64": field_errors_vs_oracle(wl, tau, f_orc, lams, "fp64")}
        if r32:
            errs["fp32"] = field_errors_vs_oracle(wl, tau, f_orc, lams, "fp32")
        out["err_vs_oracle"] = errs
        log("err_vs_oracle", errs)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
