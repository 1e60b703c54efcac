"""GPU checks of the 3D workloads at the sizes the benchmark runs.

256^3 bubbles (FP32 form with the viscous part, and FP64): one step of the
oracle is affordable on the host (about half a minute), so the whole field
is compared after one step, with the oracle's schedule frozen into the GPU
run (heat and viscous bounds), at the usual bars: FP64 1e-12, FP32 form
1e-5 per field (max-norm, relative).

512^3 interface (x walls, contrast 100): one step against the oracle's whole
fields the same way (the oracle's step takes under a minute with the box's
cores), and two steps held to properties that hold at any size and are exact
for the method: the heat step conserves the energy sum_cells C T (no
sources, adiabatic walls), keeps T within the initial bounds (maximum
principle of the LIM pass with its final stage), and the FP32 form agrees
with the FP64 path within the FP32 form's bar.
"""
import numpy as np
import pytest

from paper_2106_00282_amd import workloads as W
from _cases import make_solver, oracle_dt, rel_err, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_bubbles3d_256_one_step_vs_oracle():
    """The 256^3 bubbles benchmark workload (20 bubbles, T^2 laws, viscous
    part): one step of heat and viscous part in FP64 and in the FP32 form,
    whole fields against the oracle."""
    from oracle import oracle as orc
    wl = W.bubbles3d(256)
    tau, _ = oracle_dt(orc, wl)
    print("case bubbles3d 256^3: oracle step", flush=True)
    fo, ro = run_oracle(orc, wl, tau, 1)
    frozen = [r["lambda_G"] for r in ro]
    fields = ("T1", "T2", "alpha2", "u", "v", "w")
    for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        print(f"case bubbles3d 256^3 {precision}", flush=True)
        fg, rg, s = run_gpu(wl, tau, 1, precision=precision, frozen=frozen)
        assert [r["P"] for r in rg] == [r["P"] for r in ro]
        assert [r["visc_P"] for r in rg] == [r["visc_P"] for r in ro]
        errs = {k: rel_err(fg[k], fo[k]) for k in fields}
        print(f"per-field error vs the FP64 oracle ({precision}): {errs}", flush=True)
        for k, e in errs.items():
            assert e <= tol, (precision, k, e)
        s.close()
    # the step is not trivial: heat moved and the velocity diffused
    assert rel_err(fo["T1"], wl["fields"]["T1"]) > 1e-3
    assert rel_err(fo["u"], wl["fields"]["u"]) > 1e-4


@pytest.mark.timeout(600)
def test_interface3d_512_full_size_properties():
    """The 512^3 interface workload, two steps in FP64 and in the FP32 form
    (the FP32 run with the FP64 run's schedule): energy conserved, T within
    the initial bounds, and the two precisions within the FP32 form's bar."""
    wl = W.interface3d(512)
    f0 = wl["fields"]
    C = f0["m1"] * wl["phases"][0]["cv"] + f0["m2"] * wl["phases"][1]["cv"]
    assert wl["phases"][0]["pinf"] == wl["phases"][1]["pinf"]  # C fixed within the step
    E0 = float((C * f0["T1"]).sum())
    lo, hi = float(f0["T1"].min()), float(f0["T1"].max())
    del C
    from paper_2106_00282_amd.tlim import StepOpts
    out = {}
    sched = None
    for precision in ("fp64", "fp32"):
        print(f"case interface3d 512^3 {precision}", flush=True)
        s = make_solver(wl, precision)
        tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
        reps = []
        for k in range(2):
            fr = None if sched is None else sched[k]
            st, rep = s.advance(StepOpts(dt=tau, passes=wl["passes"], frozen_lambda=fr))
            assert st == 0
            reps.append(rep)
        if sched is None:
            sched = [r["lambda_G"] for r in reps]
            P64 = [r["P"] for r in reps]
        else:
            assert [r["P"] for r in reps] == P64
        for r in reps:
            assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-12, (precision, r["energy_before"],
                                                                          r["energy_after"])
        T = s.get_field("T1").cpu().numpy()
        out[precision] = (T, s.get_field("alpha2").cpu().numpy())
        s.close()
        # energy of the relaxed initial state against the end state (alpha2
        # and the masses are unchanged by the heat step of equal p_inf)
        E1 = float(((f0["m1"] * wl["phases"][0]["cv"] + f0["m2"] * wl["phases"][1]["cv"]) * T).sum())
        print(f"{precision}: energy change {E1 / E0 - 1:.3e}, T in [{T.min():.6f}, {T.max():.6f}] "
              f"of [{lo:.6f}, {hi:.6f}]", flush=True)
        assert abs(E1 / E0 - 1) < 1e-12
        # the FP32 form's stages carry its 1e-5 bar into the bound
        mp = 1e-12 if precision == "fp64" else 1e-5
        assert T.min() >= lo * (1 - mp) and T.max() <= hi * (1 + mp)
        del T
    e_T = rel_err(out["fp32"][0], out["fp64"][0])
    e_a = rel_err(out["fp32"][1], out["fp64"][1])
    print(f"FP32 form vs FP64 at 512^3 after 2 steps: T {e_T:.2e}, alpha2 {e_a:.2e}", flush=True)
    assert e_T <= 1e-5 and e_a <= 1e-5
    # the run is not trivial: heat moved
    assert rel_err(out["fp64"][0], f0["T1"]) > 1e-3


@pytest.mark.timeout(900)
def test_interface3d_512_one_step_vs_oracle():
    """The 512^3 interface workload itself: one step in the FP32 form (the
    benchmark's arithmetic) and in FP64 against the oracle's whole fields,
    with the oracle's schedule frozen into both runs."""
    from oracle import oracle as orc
    wl = W.interface3d(512)
    tau, _ = oracle_dt(orc, wl)
    print("case interface3d 512^3: oracle step", flush=True)
    fo, ro = run_oracle(orc, wl, tau, 1)
    frozen = [r["lambda_G"] for r in ro]
    for precision, tol in (("fp32", 1e-5), ("fp64", 1e-12)):
        print(f"case interface3d 512^3 {precision}", flush=True)
        fg, rg, s = run_gpu(wl, tau, 1, precision=precision, frozen=frozen)
        s.close()
        assert [r["P"] for r in rg] == [r["P"] for r in ro]
        errs = {k: rel_err(fg[k], fo[k]) for k in ("T1", "T2", "alpha2")}
        print(f"per-field error vs the FP64 oracle ({precision}): {errs}", flush=True)
        for k, e in errs.items():
            assert e <= tol, (precision, k, e)
        del fg
    assert rel_err(fo["T1"], wl["fields"]["T1"]) > 1e-3
