"""GPU parity on 3D grids several x tiles wide.

The 3D kernels give each wave 64 x cells; the cells at the ends of a wave
take their x neighbours from the next tile (or across the periodic wrap, or
not at all at a wall).  These grids have 3 x tiles with a ragged last one
(160 = 64 + 64 + 32, 130 = 64 + 64 + 2), y rows that do not fill the last
row block, and both boundary kinds in x, so every halo case of the stage,
coefficient and viscous kernels is compared with the oracle.  Same bars as
everywhere: FP64 1e-12, FP32 form 1e-5 per field (max-norm, relative).
"""
import numpy as np
import pytest

from paper_2106_00282_amd import workloads as W
from _cases import make_solver, oracle_dt, rel_err, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _bubbles(shape, walls):
    wl = W.bubbles3d(shape[0], shape=shape)
    for c in "uvw":  # a stronger flow, so that the viscous heating shows
        wl["fields"][c] = np.ascontiguousarray(30.0 * wl["fields"][c])
    if walls:
        wl["bc"] = (W.ADIABATIC, W.PERIODIC, W.ADIABATIC)
    return wl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(160, 36, 22), (130, 20, 9)])
def test_bubbles3d_wide_heat_viscous_heating(shape, walls, precision):
    """Heat conduction, the viscous part and its heating of the phases, two
    steps, against the oracle with its schedule frozen into both sides."""
    from oracle import oracle as orc
    wl = _bubbles(shape, walls)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2, visc_heating=1)
    print(f"case bubbles3d {shape} walls={walls} {precision}", flush=True)
    fg, rg, s = run_gpu(wl, tau, 2, precision=precision, frozen=[r["lambda_G"] for r in ro], visc_heating=1)
    assert [r["visc_P"] for r in rg] == [r["visc_P"] for r in ro]
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    tol = 1e-12 if precision == "fp64" else 1e-5
    errs = {k: rel_err(fg[k], fo[k]) for k in ("T1", "T2", "alpha2", "u", "v", "w")}
    print(f"per-field error vs the FP64 oracle: {errs}")
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)
    # the run is not trivial: heat moved and the velocity diffused
    assert rel_err(fo["T1"], wl["fields"]["T1"]) > 1e-3
    assert rel_err(fo["u"], wl["fields"]["u"]) > 1e-4
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_interface3d_c5_shape_forward(precision):
    """The 512^3 interface workload's setup (x adiabatic, y and z periodic,
    conductivity contrast 100, 12 modes of amplitude 5 cells) on a
    192 x 64 x 48 box, three steps against the oracle."""
    from oracle import oracle as orc
    wl = W.interface3d(192, shape=(192, 64, 48))
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 3)
    print(f"case interface3d 192x64x48 {precision}", flush=True)
    fg, rg, s = run_gpu(wl, tau, 3, precision=precision, frozen=[r["lambda_G"] for r in ro])
    tol = 1e-12 if precision == "fp64" else 1e-5
    errs = {k: rel_err(fg[k], fo[k]) for k in ("T1", "T2", "alpha2")}
    print(f"per-field error vs the FP64 oracle: {errs}")
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)
    assert rel_err(fo["T1"], wl["fields"]["T1"]) > 1e-3
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_interface3d_c5_shape_adjoint_checkpoints_every_2(precision):
    """Forward with checkpoints every 2 steps and the adjoint on the c5
    setup (192 x 64 x 48, 4 steps), against the oracle's adjoint with the
    run's own schedule.  In an FP64 context the checkpoints are the FP64
    trajectory (1e-12).  In an FP32 context the forward runs the FP32 form
    and the adjoint recomputes and reverses in FP64 from its checkpoints:
    T^0 is exact and T^2 carries the FP32 form's error, so the gradient is
    held to the FP32 bar (1e-5)."""
    import torch
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.interface3d(192, shape=(192, 64, 48))
    tau, _ = oracle_dt(orc, wl)
    steps = 4
    print(f"case interface3d adjoint 192x64x48 {precision}", flush=True)
    s = make_solver(wl, precision)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 2)
    assert ckpt.shape[0] == 2
    TN = s.get_field("T1").cpu().numpy()
    rng = np.random.default_rng(21)
    w = rng.standard_normal(TN.shape)
    dT0, dk0 = s.adjoint(opts, steps, 2, ckpt, lam, torch.from_numpy(w))
    f = wl["fields"]
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"],
                                       orc.StepOpts(tau=tau, passes=3), steps, np.array(lam), f["alpha2"],
                                       f["m1"], f["m2"], f["T1"], w)
    tol = 1e-12 if precision == "fp64" else 1e-5
    e_T, e_g = rel_err(TN, oTN), rel_err(dT0.cpu().numpy(), odT0)
    e_k = [abs(dk0[k] / odk0[k] - 1) for k in range(2)]
    print(f"T^N {e_T:.2e}, dL/dT0 {e_g:.2e}, dL/dk0 {e_k}")
    assert e_T <= tol and e_g <= tol
    # dL/dk0 sums over every cell and pass with cancellation (see the 2D
    # adjoint tests): 1e-10 in FP64
    for k in range(2):
        assert e_k[k] <= (1e-10 if precision == "fp64" else 1e-5), (k, e_k)
    s.close()
