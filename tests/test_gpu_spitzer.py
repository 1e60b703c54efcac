"""GPU parity of the Spitzer-Harm conductivity law (Sec. 4.4): lambda =
k0 (T/T0)^n / ln Lambda_ei(rho, T) with the two-branch Coulomb logarithm
floored at 1, against the FP64 oracle on the same seeded inputs.

The workloads put cells on both branches and on the floor (the oracle pins
check that).  Tolerances as for the power law: FP64 <= 1e-12 relative per
field, FP32 form <= 1e-5, adjoint vs the oracle adjoint <= 1e-12 (the dL/dk0
sums 1e-10).
"""
import numpy as np
import pytest

from paper_2106_00282_amd import workloads as W
from _cases import oracle_dt, rel_err, run_gpu, run_oracle, make_solver

pytestmark = pytest.mark.gpu

FIELDS_T = ("T1", "T2", "alpha2")


def _frozen(reps):
    return [r["lambda_G"] for r in reps]


def _cut(wl, nx, ny, ng):
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    return wl


def test_spitzer_levelset2d_full_size_fp64():
    """1024^2, 10 steps x 3 passes at 200x: the first step as one launch with
    P on the device, then predicted steps whose last launch builds the next
    step's start; and the same run with every step one launch."""
    from oracle import oracle as orc
    wl = W.levelset2d_spitzer(1024)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 10)
    fg, rg, _ = run_gpu(wl, tau, 10)
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
    print("spitzer 1024^2 fp64 errors", errs, "P", rg[0]["P"])
    assert max(errs.values()) <= 1e-12, errs
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-13
    assert rg[0]["sweep_launches"] == 1
    assert sum(r["predicted"] for r in rg[1:]) >= 5
    fw, rw, _ = run_gpu(wl, tau, 10, whole_step=1)
    assert [r["P"] for r in rw] == [r["P"] for r in ro]
    assert max(rel_err(fw[k], fo[k]) for k in FIELDS_T) <= 1e-12


@pytest.mark.parametrize("shape", [(260, 150), (90, 331), (67, 1)])
def test_spitzer_levelset2d_ragged(shape):
    """Ragged grids (64- and 128-row tiles, a 1-row grid), FP64 at 1e-12 and
    the FP32 form at 1e-5, 2 steps with the oracle's schedule."""
    from oracle import oracle as orc
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = _cut(W.levelset2d_spitzer(ng), nx, ny, ng)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, _, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    assert max(rel_err(fg[k], fo[k]) for k in FIELDS_T) <= 1e-12
    f32, _, _ = run_gpu(wl, tau, 2, precision="fp32", frozen=_frozen(ro))
    assert max(rel_err(f32[k], fo[k]) for k in ("T1", "T2")) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_spitzer_bubbles3d_with_viscous(precision):
    """3D bubbles with the viscous part and Spitzer-Harm heat conduction."""
    from oracle import oracle as orc
    wl = W.bubbles3d(40)
    wl["phases"] = W.spitzer_phases(wl["phases"])
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:33, :36, :])
    wl["n"] = (40, 36, 33)
    wl["h"] = (1 / 40, 1 / 40, 1 / 40)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, _, _ = run_gpu(wl, tau, 2, precision=precision, frozen=_frozen(ro))
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert max(rel_err(fg[k], fo[k]) for k in ("T1", "T2", "u", "v", "w")) <= tol


@pytest.mark.parametrize("case", ["blocked2d", "grid3d"])
def test_spitzer_adjoint_vs_oracle(case):
    """The adjoint through the Spitzer-Harm law (the blocked 2D reverse
    kernel's pass epilogue, and the per-cell kernel on a 3D grid) against
    the oracle adjoint, with the run's schedule."""
    import torch
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    if case == "grid3d":
        wl = W.bubbles3d(20)
        wl["viscous"] = False
        for k in ("u", "v", "w"):
            wl["fields"].pop(k)
        wl["phases"] = W.spitzer_phases(wl["phases"])
    else:
        wl = W.levelset2d_spitzer(64)
    tau, _ = oracle_dt(orc, wl)
    steps = 3
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    TN = s.get_field("T1").cpu().numpy()
    rng = np.random.default_rng(15)
    Tstar = wl["fields"]["T1"] * (1 + 0.05 * rng.standard_normal(TN.shape))
    dT0, dk0 = s.adjoint(opts, steps, 1, ckpt, lam, torch.from_numpy(TN - Tstar))
    f = wl["fields"]
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"],
                                       orc.StepOpts(tau=tau, passes=3), steps, np.array(lam), f["alpha2"],
                                       f["m1"], f["m2"], f["T1"], TN - Tstar)
    assert rel_err(TN, oTN) < 1e-12
    assert rel_err(dT0.cpu().numpy(), odT0) < 1e-12
    for k in range(2):
        assert dk0[k] == pytest.approx(odk0[k], rel=1e-10)


def test_spitzer_invalid_constants_rejected():
    from paper_2106_00282_amd.tlim import E_ARG, TlimError
    wl = W.levelset2d_spitzer(16)
    s = make_solver(wl)
    bad = [dict(sh_D=0.0), dict(sh_LD=-1.0), dict(sh_LD=0.0, sh_dB=0.0), dict(sh_dB=float("inf")),
           dict(law=7)]
    for b in bad:
        p = dict(wl["phases"][0])
        p.update(b)
        with pytest.raises(TlimError) as ei:
            s.set_phase(0, p)
        assert ei.value.status == E_ARG, b
    # a power-law phase ignores the length constants
    p = dict(wl["phases"][0])
    p.update(law=W.LAW_POWER, sh_D=0.0)
    s.set_phase(0, p)


@pytest.mark.parametrize("sources", [False, True])
def test_spitzer_unequal_pinf_and_sources(sources):
    """The Spitzer-Harm law on stiffened-gas phases (p_inf 6e8 / 0) out of
    thermal equilibrium, with and without heat sources: relaxation, C_eff,
    the alpha_2 update and (with sources) the tiled coefficient kernel with
    the law's logarithms, against the oracle."""
    from oracle import oracle as orc
    nx, ny = 70, 48
    rng = np.random.default_rng(17)
    ph = [dict(gamma=4.4, pinf=6e8, cv=1606.0, q=0.0, k0=0.6, T0=300.0, npow=2.5, mu=0.0),
          dict(gamma=1.4, pinf=0.0, cv=714.0, q=0.0, k0=0.03, T0=300.0, npow=2.5, mu=0.0)]
    # lengths chosen so that T ~ 300 and rho ~ 1..1e3 straddle the branch
    # point (T = (sh_LD/sh_dB)^2 = 300) and the floor
    ph = W.spitzer_phases(ph, sh_D=0.25, sh_LD=300.0 ** 0.5, sh_dB=1.0, npow=2.5)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    a1 = 0.5 * (1 - np.tanh((x[None, :] - 0.5 - 0.1 * np.sin(2 * np.pi * y[:, None])) / (2.0 / nx)))
    a2 = 1 - a1
    rho1 = (1e9 + 6e8) / (3.4 * 1606.0 * 293.0)
    rho2 = 1e5 / (0.4 * 714.0 * 293.0)
    T1 = 280.0 + 40 * rng.random((ny, nx))
    T2 = 280.0 + 40 * rng.random((ny, nx))
    fields = dict(alpha2=a2.reshape(1, ny, nx), m1=(a1 * rho1).reshape(1, ny, nx),
                  m2=(a2 * rho2).reshape(1, ny, nx), T1=T1.reshape(1, ny, nx), T2=T2.reshape(1, ny, nx))
    if sources:
        fields.update(src1=1e3 * rng.random((1, ny, nx)), src2=1e2 * rng.random((1, ny, nx)))
    fields = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}
    wl = dict(n=(nx, ny, 1), h=(1e-3, 1e-3, 1.0), bc=(0, 1, 0), phases=ph, fields=fields, dt_factor=50.0,
              passes=3, viscous=False)
    # the law's three regimes are present in the input
    T = fields["T1"]
    rho = fields["m1"] + fields["m2"]
    L = np.log(0.25 * np.sqrt(T / rho) / np.maximum(300.0 ** 0.5 / T, 1.0 / np.sqrt(T)))
    assert (L < 1).any() and ((L > 1) & (T < 300)).any() and ((L > 1) & (T > 300)).any()
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
    assert max(errs.values()) <= 1e-12, errs


def test_spitzer_levelset2d_full_size_fp32():
    """The FP32 form on the 1024^2 Spitzer-Harm workload, 10 steps, per-field
    error against the FP64 oracle (with the oracle's schedule)."""
    from oracle import oracle as orc
    wl = W.levelset2d_spitzer(1024)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 10)
    fg, rg, _ = run_gpu(wl, tau, 10, precision="fp32", frozen=_frozen(ro))
    errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
    print("spitzer 1024^2 fp32 errors", errs)
    assert errs["T1"] <= 1e-5 and errs["T2"] <= 1e-5 and errs["alpha2"] <= 1e-12
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-12
