"""Shared drivers for the parity tests: run a workload through the oracle
and through the GPU library on the same seeded inputs."""
from __future__ import annotations

import numpy as np

from paper_2106_00282_amd import workloads as W


def oracle_dt(orc, wl, eps=1e-10):
    """tau = dt_factor * 2 / lambda_G of the initial post-relaxation state,
    evaluated by the oracle (the explicit limit is 2/lambda_G)."""
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    f = {k: v.copy() for k, v in wl["fields"].items()}
    orc.relax(g, wl["phases"], f["alpha2"], f["m1"], f["m2"], f["T1"], f["T2"], eps)
    Lam = orc.cell_conductivity(g, wl["phases"], f["alpha2"], f["T1"], f["m1"], f["m2"])
    Cap = orc.heat_capacity(g, wl["phases"], f["alpha2"], f["m1"], f["m2"], f["T1"], eps)
    lam = orc.gershgorin(g, Lam, Cap)
    return wl["dt_factor"] * 2.0 / lam, lam


def run_oracle(orc, wl, tau, steps, passes=None, viscous=None, frozen=None, **kw):
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    f = {k: v.copy() for k, v in wl["fields"].items()}
    opts = orc.StepOpts(tau=tau, passes=passes or wl["passes"],
                        do_viscous=int(wl.get("viscous", False) if viscous is None else viscous), **kw)
    reps = []
    for s in range(steps):
        fl = None if frozen is None else frozen[s]
        st, rep = orc.step(g, wl["phases"], opts, f, frozen_lambda=fl)
        reps.append(rep)
    return f, reps


def make_solver(wl, precision="fp64"):
    from paper_2106_00282_amd.tlim import Solver
    s = Solver(wl["n"], wl["h"], wl["bc"], precision=precision)
    s.set_workload(wl)
    return s


def run_gpu(wl, tau, steps, precision="fp64", passes=None, viscous=None, frozen=None, **kw):
    from paper_2106_00282_amd.tlim import StepOpts
    s = make_solver(wl, precision)
    reps = []
    for k in range(steps):
        o = StepOpts(dt=tau, passes=passes or wl["passes"],
                     do_viscous=int(wl.get("viscous", False) if viscous is None else viscous),
                     frozen_lambda=None if frozen is None else frozen[k], **kw)
        st, rep = s.advance(o)
        assert st == 0, (st, rep)
        reps.append(rep)
    out = {k: s.get_field(k).cpu().numpy() for k in wl["fields"]}
    return out, reps, s


def rel_err(a, b):
    """max |a - b| / max |b| (max-norm relative error of a field)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))
