"""GPU parity: the HIP path against the FP64 oracle on the same seeded
inputs, through the C ABI.

Tolerances: FP64 path <= 1e-12 relative (max-norm per field); FP32 form
<= 1e-5 relative per field; adjoint vs oracle adjoint <= 1e-12, vs central
finite differences <= 1e-6.  The schedule (lambda_max per pass) is the
oracle's, frozen into both sides, wherever a test compares several passes,
so that P (an integer decided in floating point) is decided once.
"""
import numpy as np
import pytest

from paper_2106_00282_amd import workloads as W
from _cases import oracle_dt, rel_err, run_gpu, run_oracle, make_solver

pytestmark = pytest.mark.gpu

FIELDS_T = ("T1", "T2", "alpha2")


def _frozen(reps):
    return [r["lambda_G"] for r in reps]


def _compare(fo, fg, names, tol):
    errs = {k: rel_err(fg[k], fo[k]) for k in names}
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)
    return errs


# ----------------------------------------------------------------- FP64 path

@pytest.mark.parametrize("seed", list(range(16)))
def test_random_small_cases_vs_oracle(seed):
    """Property-style sweep: random 1D/2D/3D grids, boundary conditions,
    phase constants and out-of-equilibrium states (workloads.random_case),
    2 steps in FP64 against the oracle at 1e-12 (schedule frozen to the
    oracle's), and every fourth case also in the FP32 form at 1e-5."""
    from oracle import oracle as orc
    wl = W.random_case(seed)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    print("case", seed, wl["n"], wl["bc"], "passes", wl["passes"], "dt x", round(wl["dt_factor"], 1))
    _compare(fo, fg, FIELDS_T, 1e-12)
    if seed % 4 == 0:
        f32, _, _ = run_gpu(wl, tau, 2, precision="fp32", frozen=_frozen(ro))
        _compare(fo, f32, ("T1", "T2"), 1e-5)


def test_heat1d_fp64_single_step():
    """1024 cells, one step at 100x the explicit limit: P = 12, 23 sweeps."""
    from oracle import oracle as orc
    wl = W.heat1d()
    tau, lam = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 1)
    fg, rg, s = run_gpu(wl, tau, 1)
    assert rg[0]["P"] == ro[0]["P"] == [12]
    assert rg[0]["lambda_G"][0] == pytest.approx(ro[0]["lambda_G"][0], rel=1e-14)
    _compare(fo, fg, FIELDS_T, 1e-12)
    assert abs(rg[0]["energy_after"] / rg[0]["energy_before"] - 1) < 1e-14


@pytest.mark.parametrize("shape", [(100, 76), (64, 4), (67, 1), (3, 130), (260, 150), (90, 331)])
def test_levelset2d_fp64_ragged(shape):
    """Reduced level-set workload on grids that span several tiles and leave
    ragged tails (64- and 128-row blocked tiles); 2 steps x 3 Picard passes."""
    from oracle import oracle as orc
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = W.levelset2d(ng)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
        assert wl["fields"][k].shape == (1, ny, nx)
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    _compare(fo, fg, FIELDS_T, 1e-12)


@pytest.mark.parametrize("precision,shape,bc", [("fp64", (261, 140), "periodic"), ("fp64", (129, 128), "adiabatic"),
                                                ("fp64", (300, 200), "adiabatic"), ("fp32", (261, 140), "periodic"),
                                                ("fp32", (129, 128), "adiabatic"), ("fp32", (300, 200), "adiabatic"),
                                                ("fp32", (260, 150), "periodic"), ("fp32", (128, 128), "periodic"),
                                                ("fp32", (130, 256), "adiabatic")])
def test_two_cells_per_lane_tiles(precision, shape, bc):
    """The FP32 form's float stages run 128-wide tiles with two cells per
    lane on grids of at least 128 x 128 cells (even widths when x is
    periodic, so that no lane's pair straddles the wrap): an odd periodic
    width (which keeps one cell per lane), the smallest such grid (a
    one-column last tile), and adiabatic walls on both axes, where the pairs
    past the walls are clamped copies; the FP64 path (64 x 128 tiles) on the
    same grids.  2 steps x 3 passes against the oracle (FP64 1e-12, FP32
    form 1e-5)."""
    from oracle import oracle as orc
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = W.levelset2d(ng)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    if bc == "adiabatic":
        wl["bc"] = (W.ADIABATIC, W.ADIABATIC, W.PERIODIC)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, precision=precision, frozen=_frozen(ro))
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    if precision == "fp64":
        _compare(fo, fg, FIELDS_T, 1e-12)
    else:
        errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
        print("fp32 two-cells-per-lane per-field error:", shape, bc, errs)
        assert max(errs.values()) <= 1e-5
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-12


@pytest.mark.parametrize("precision,shape", [("fp64", (150, 140)), ("fp32", (150, 140)), ("fp32", (100, 76))])
def test_power_law_with_a_general_exponent(precision, shape):
    """A power law whose exponent the law evaluation does not write out as
    products (n = 1.7 in one phase: the general power) on grids of the
    blocked 2D kernels, against the oracle (2 steps x 3 passes)."""
    from oracle import oracle as orc
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = W.levelset2d(ng)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    wl["phases"] = [dict(p) for p in wl["phases"]]
    wl["phases"][1]["npow"] = 1.7
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, precision=precision, frozen=_frozen(ro))
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    if precision == "fp64":
        _compare(fo, fg, FIELDS_T, 1e-12)
    else:
        errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
        assert max(errs.values()) <= 1e-5, errs


def test_levelset2d_fp64_full_size():
    """1024^2 periodic, T^2 conductivities, 10 steps x 3 passes at 200x the
    explicit limit (the benchmark workload) against the full oracle run."""
    from oracle import oracle as orc
    wl = W.levelset2d(1024)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 10)
    fg, rg, _ = run_gpu(wl, tau, 10)
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    _compare(fo, fg, FIELDS_T, 1e-12)
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-13
    # the first step (no schedule history) runs as one launch that decides P
    # on the device; after it the schedule is predicted and confirmed without
    # a readback per pass
    assert rg[0]["sweep_launches"] == 1 and not rg[0]["predicted"]
    assert sum(r["predicted"] for r in rg[1:]) >= 5
    # the same run as one launch per step, P decided on the device
    fw, rw, _ = run_gpu(wl, tau, 10, whole_step=1)
    assert [r["P"] for r in rw] == [r["P"] for r in ro]
    assert all(r["sweep_launches"] == 1 for r in rw)
    _compare(fo, fw, FIELDS_T, 1e-12)


@pytest.mark.parametrize("shape,bc", [((256, 256), "periodic"), ((300, 200), "adiabatic"),
                                      ((70, 390), "periodic"), ((1000, 131), "adiabatic")])
def test_whole_step_kernel_vs_oracle(shape, bc):
    """FP64 2D heat steps whose schedule is decided on the device: one
    cooperative launch per step (relaxation, every Picard pass with its P
    from the reduced lambda_G, stages in blocks with ring exchanges),
    against the oracle deciding its own P (3 steps x 3 passes), then the
    same steps pipelined without reports."""
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = W.levelset2d(ng)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    if bc == "adiabatic":
        wl["bc"] = (W.ADIABATIC, W.ADIABATIC, W.PERIODIC)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 3)
    fg, rg, _ = run_gpu(wl, tau, 3, whole_step=1)
    assert [r["P"] for r in rg] == [r["P"] for r in ro]
    assert all(r["sweep_launches"] == 1 for r in rg), [r["sweep_launches"] for r in rg]
    # never: the first step reads P back pass by pass
    fn, rn, _ = run_gpu(wl, tau, 3, whole_step=2)
    assert [r["P"] for r in rn] == [r["P"] for r in ro]
    assert rn[0]["sweep_launches"] > 1
    _compare(fo, fn, FIELDS_T, 1e-12)
    assert all(r["sweeps"] == sum(2 * p - 1 for p in r["P"]) for r in rg)
    _compare(fo, fg, FIELDS_T, 1e-12)
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-13
    s = make_solver(wl)
    for _ in range(3):
        assert s.advance(StepOpts(dt=tau, passes=wl["passes"], whole_step=1), report=False)[0] == 0
    s.finish()
    assert rel_err(s.get_field("T1").cpu().numpy(), fo["T1"]) < 1e-12


def test_bubbles3d_fp64_with_viscous():
    """3D periodic bubbles, heat + viscous sub-step, on a 40x36x33 grid."""
    from oracle import oracle as orc
    wl = W.bubbles3d(40)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:33, :36, :])
    wl["n"] = (40, 36, 33)
    wl["h"] = (1 / 40, 1 / 40, 1 / 40)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    assert [r["visc_P"] for r in rg] == [r["visc_P"] for r in ro]
    _compare(fo, fg, FIELDS_T + ("u", "v", "w"), 1e-12)


@pytest.mark.parametrize("precision,walls", [("fp64", False), ("fp64", True), ("fp32", False)])
def test_viscous_heating_vs_oracle(precision, walls):
    """Viscous part with the phase heating (Sec. 3.2, phase internal
    energies) on 3D bubbles with a 30x stronger velocity, periodic or with
    adiabatic walls in x and z: temperatures, volume fraction and velocity
    after 2 steps against the oracle; the heating itself must be visible."""
    from oracle import oracle as orc
    wl = W.bubbles3d(40)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:33, :36, :])
    for c in "uvw":
        wl["fields"][c] = np.ascontiguousarray(30.0 * wl["fields"][c])
    wl["n"] = (40, 36, 33)
    wl["h"] = (1 / 40, 1 / 40, 1 / 40)
    if walls:
        wl["bc"] = (W.ADIABATIC, W.PERIODIC, W.ADIABATIC)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2, visc_heating=1)
    fn, _ = run_oracle(orc, wl, tau, 2)
    assert rel_err(fo["T1"], fn["T1"]) > 1e-4  # the heating changes T
    fg, rg, _ = run_gpu(wl, tau, 2, precision=precision, frozen=_frozen(ro), visc_heating=1)
    assert [r["visc_P"] for r in rg] == [r["visc_P"] for r in ro]
    _compare(fo, fg, FIELDS_T + ("u", "v", "w"), 1e-12 if precision == "fp64" else 1e-5)


def _with_total_energy(wl):
    """Add rho E = sum_k (m_k C_v,k T_k + alpha_k p_inf,k) + rho |u|^2 / 2."""
    f = wl["fields"]
    ph = wl["phases"]
    a2 = f["alpha2"]
    E = (f["m1"] * ph[0]["cv"] * f["T1"] + (1 - a2) * ph[0]["pinf"] + f["m2"] * ph[1]["cv"] * f["T2"]
         + a2 * ph[1]["pinf"])
    E = E + 0.5 * (f["m1"] + f["m2"]) * sum(f[c] ** 2 for c in "uvw" if c in f)
    f["E"] = np.ascontiguousarray(E)
    return f["E"].copy()


@pytest.mark.parametrize("precision,walls", [("fp64", False), ("fp64", True), ("fp32", True)])
def test_total_energy_viscous_and_heat_vs_oracle(precision, walls):
    """Total energy through 2 steps of 3D bubbles with the viscous part
    (work of the viscous flux with the predicted velocity) and heat
    conduction (flux divergence of the last pass), 30x stronger velocity:
    E and its change against the oracle."""
    from oracle import oracle as orc
    wl = W.bubbles3d(40)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:33, :36, :])
    for c in "uvw":
        wl["fields"][c] = np.ascontiguousarray(30.0 * wl["fields"][c])
    wl["n"] = (40, 36, 33)
    wl["h"] = (1 / 40, 1 / 40, 1 / 40)
    if walls:
        wl["bc"] = (W.ADIABATIC, W.PERIODIC, W.ADIABATIC)
    E0 = _with_total_energy(wl)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2, visc_heating=1)
    fg, rg, _ = run_gpu(wl, tau, 2, precision=precision, frozen=_frozen(ro), visc_heating=1)
    tol = 1e-12 if precision == "fp64" else 1e-5
    _compare(fo, fg, FIELDS_T + ("u", "v", "w", "E"), tol)
    dEo, dEg = fo["E"] - E0, fg["E"] - E0
    assert np.abs(dEo).max() > 1e-6 * np.abs(E0).max()
    assert rel_err(dEg, dEo) < (1e-9 if precision == "fp64" else 1e-2)
    if not walls:
        # periodic, no sources: the total energy is conserved
        assert abs(dEg.sum()) < 1e-9 * np.abs(dEg).sum()


@pytest.mark.parametrize("case", ["levelset_fp64", "levelset_fp32", "sg_sources"])
def test_total_energy_heat_only_vs_oracle(case):
    """Heat steps with the total energy: the fused 2D path (relaxation with
    the first coefficients, next-pass coefficients in the last launch) in
    both precisions, and the general stiffened-gas step with heat sources;
    clearing E stops its update."""
    from oracle import oracle as orc
    if case == "sg_sources":
        rng = np.random.default_rng(11)
        nx, ny = 48, 40
        ph = [dict(gamma=4.4, pinf=6e8, cv=1606.0, q=0.0, k0=0.6, T0=300.0, npow=1.0, mu=0.0),
              dict(gamma=1.4, pinf=0.0, cv=714.0, q=0.0, k0=0.03, T0=300.0, npow=1.0, mu=0.0)]
        x = (np.arange(nx) + 0.5) / nx
        y = (np.arange(ny) + 0.5) / ny
        a1 = 0.5 * (1 - np.tanh((x[None, :] - 0.5 - 0.1 * np.sin(2 * np.pi * y[:, None])) / (2.0 / nx)))
        rho1 = (1e9 + 6e8) / (3.4 * 1606.0 * 293.0)
        rho2 = 1e5 / (0.4 * 714.0 * 293.0)
        fields = dict(alpha2=1 - a1, m1=a1 * rho1, m2=(1 - a1) * rho2, T1=293.0 + 20 * rng.random((ny, nx)),
                      T2=293.0 + 20 * rng.random((ny, nx)), src1=1e9 * rng.random((ny, nx)),
                      src2=1e8 * rng.random((ny, nx)))
        fields = {k: np.ascontiguousarray(v.reshape(1, ny, nx), dtype=np.float64) for k, v in fields.items()}
        wl = dict(n=(nx, ny, 1), h=(1e-3, 1e-3, 1.0), bc=(0, 1, 0), phases=ph, fields=fields, dt_factor=50.0,
                  passes=3, viscous=False)
        precision = "fp64"
    else:
        wl = W.levelset2d(96)
        precision = case.split("_")[1]
    E0 = _with_total_energy(wl)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 3)
    fg, rg, s = run_gpu(wl, tau, 3, precision=precision, frozen=_frozen(ro))
    tol = 1e-12 if precision == "fp64" else 1e-5
    _compare(fo, fg, FIELDS_T + ("E",), tol)
    dEo, dEg = fo["E"] - E0, fg["E"] - E0
    assert np.abs(dEo).max() > 1e-6 * np.abs(E0).max()
    assert rel_err(dEg, dEo) < (1e-9 if precision == "fp64" else 1e-2)
    from paper_2106_00282_amd.tlim import StepOpts, TlimError
    s.clear_field("E")
    st, _ = s.advance(StepOpts(dt=tau, passes=wl["passes"]))
    assert st == 0
    with pytest.raises(TlimError):
        s.get_field("E")
    with pytest.raises(TlimError):
        s.clear_field("T1")


def test_interface3d_fp64_adiabatic_x():
    from oracle import oracle as orc
    wl = W.interface3d(32, nmodes=12)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    _compare(fo, fg, FIELDS_T, 1e-12)


def test_mispredicted_schedule_rolls_back():
    """Change k0 between steps so that the predicted P is wrong: the step is
    rolled back, rerun with one readback per pass, and still matches the
    oracle run with the same change.  Prediction resumes once the new
    schedule has held for a step."""
    from oracle import oracle as orc
    wl = W.levelset2d(96)
    tau, _ = oracle_dt(orc, wl)
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    fo = {k: v.copy() for k, v in wl["fields"].items()}
    s = make_solver(wl)
    from paper_2106_00282_amd.tlim import StepOpts
    ph = [dict(p) for p in wl["phases"]]
    reps = []
    for step, scale in enumerate((1.0, 1.0, 1.0, 4.0, 4.0, 4.0)):
        for k in range(2):
            ph[k]["k0"] = wl["phases"][k]["k0"] * scale
            s.set_phase(k, ph[k])
        orc.step(g, ph, orc.StepOpts(tau=tau, passes=3), fo)
        st, rep = s.advance(StepOpts(dt=tau, passes=3))
        assert st == 0
        reps.append(rep)
    # steps 0 and 1 build the history, step 2 is predicted; the new k0 of
    # step 3 makes its prediction miss, step 4 runs with one readback per
    # pass (the schedule changed) and step 5 is predicted again
    assert reps[2]["predicted"]
    assert reps[3]["mispredicted"] and not reps[3]["predicted"]
    assert not reps[4]["predicted"] and not reps[4]["mispredicted"]
    assert reps[5]["predicted"]
    assert reps[3]["sweeps"] == sum(2 * p - 1 for p in reps[3]["P"])
    assert rel_err(s.get_field("T1").cpu().numpy(), fo["T1"]) < 1e-12


@pytest.mark.parametrize("precision,n,hot,miss,whole", [("fp64", 256, 1.0, False, 0), ("fp64", 192, 3.0, True, 0),
                                                        ("fp32", 192, 3.0, True, 0), ("fp32", 256, 3.0, False, 0),
                                                        ("fp64", 192, 3.0, True, 1)])
def test_pipelined_steps_match_oracle(precision, n, hot, miss, whole):
    """Steps without a report run pipelined (each verified by the next call).
    With a hot spot (T up to 1 + hot) lambda_G falls from step to step, so
    the P predicted from two steps back is wrong now and then and the step
    must be redone; the result must still match the oracle's unfrozen run.
    FP64 with whole = 1 runs each step as one launch that decides P itself."""
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(n)
    if hot != 1.0:
        x = (np.arange(n) + 0.5) / n
        r2 = (x[None, :] - 0.3) ** 2 + (x[:, None] - 0.6) ** 2
        bump = 1.0 + hot * np.exp(-r2 / (2 * 0.03 ** 2))
        for k in ("T1", "T2"):
            wl["fields"][k] = np.ascontiguousarray(wl["fields"][k] * bump[None])
    tau, _ = oracle_dt(orc, wl)
    steps = 8
    fo, ro = run_oracle(orc, wl, tau, steps)
    Ps = [r["P"] for r in ro]
    s = make_solver(wl, precision)
    o = StepOpts(dt=tau, passes=3, whole_step=whole)
    st, rep = s.advance(o)  # first step: synchronous, sets the schedule history
    assert st == 0 and rep["P"] == Ps[0]
    for _ in range(steps - 1):
        assert s.advance(o, report=False)[0] == 0
    assert s.finish() == 0
    fg = {k: s.get_field(k).cpu().numpy() for k in FIELDS_T}
    tol = 1e-12 if precision == "fp64" else 1e-5
    _compare(fo, fg, FIELDS_T, tol)
    if miss:
        # a pipelined step k >= 2 is predicted with the last P of step k-2
        # for every pass: here the schedule changes enough for some to miss
        assert any(Ps[k] != [Ps[k - 2][-1]] * 3 for k in range(2, steps)), Ps


@pytest.mark.parametrize("precision,whole", [("fp64", 0), ("fp32", 0), ("fp64", 1)])
def test_pipelined_dt_change_redoes_steps(precision, whole):
    """Once the schedule is steady, steps without a report run pipelined.  A
    larger dt then makes the pending step's predicted P wrong: the next call
    finds it after enqueuing its own step, redoes the pending one and reruns
    its own; a final finish() completes the last one.  Matches the oracle run
    with the same dt sequence.  The one-launch FP64 step (whole = 1) decides
    P on the device: it pipelines from the first step and redoes nothing."""
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(160)
    tau, _ = oracle_dt(orc, wl)
    dts = [tau] * 5 + [2.5 * tau] * 3 + [tau] * 2
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    fo = {k: v.copy() for k, v in wl["fields"].items()}
    s = make_solver(wl, precision)
    for dt in dts:
        orc.step(g, wl["phases"], orc.StepOpts(tau=dt, passes=3), fo)
        assert s.advance(StepOpts(dt=dt, passes=3, whole_step=whole), report=False)[0] == 0
    assert s.finish() == 0
    # one reported step reads the context's pipelining totals
    orc.step(g, wl["phases"], orc.StepOpts(tau=tau, passes=3), fo)
    st, rep = s.advance(StepOpts(dt=tau, passes=3, whole_step=whole))
    assert st == 0
    if precision == "fp64" and whole:
        assert rep["pipelined_steps"] == len(dts) and rep["pipeline_redos"] == 0, rep
    else:
        assert rep["pipelined_steps"] >= 3 and rep["pipeline_redos"] >= 1, rep
    fg = {k: s.get_field(k).cpu().numpy() for k in FIELDS_T}
    _compare(fo, fg, FIELDS_T, 1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sweep_timing_covers_the_passes_enqueued_behind_device_work(precision):
    """time_sweeps: a step's first pass follows the previous step's readback
    and is not timed; the later passes of a predicted step are, and the
    report counts their stages and launches.  Steps that read every pass's
    bound back (and the whole-step launch) time nothing."""
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(256)
    s = make_solver(wl, precision)
    tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
    reps = []
    for _ in range(5):
        st, rep = s.advance(StepOpts(dt=tau, passes=3, time_sweeps=1))
        assert st == 0
        reps.append(rep)
    s.close()
    for r in reps:
        assert 0 <= r["timed_launches"] <= r["sweep_launches"] and 0 <= r["timed_sweeps"] <= r["sweeps"]
        if r["predicted"]:
            # passes 2 and 3 are timed, pass 1 is not
            assert r["timed_sweeps"] == sum(2 * p - 1 for p in r["P"][1:])
            assert r["timed_launches"] >= 2 and r["sweep_ms"] > 0.0
        else:
            assert r["timed_sweeps"] == 0 and r["timed_launches"] == 0 and r["sweep_ms"] == 0.0
    assert sum(r["predicted"] for r in reps) >= 2


@pytest.mark.parametrize("whole", [0, 1])
def test_pipelined_step_then_report_and_phase_change(whole):
    """A pending pipelined step is completed by set_phase (which may make
    the next prediction wrong) and by a reported step; the sequence matches
    the oracle (FP64, one launch per step or per block of stages)."""
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(128)
    tau, _ = oracle_dt(orc, wl)
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    fo = {k: v.copy() for k, v in wl["fields"].items()}
    s = make_solver(wl)
    ph = [dict(p) for p in wl["phases"]]
    o = StepOpts(dt=tau, passes=3, whole_step=whole)
    for step, (scale, report) in enumerate(((1.0, True), (1.0, False), (1.0, False), (3.0, False), (3.0, False),
                                             (3.0, True), (3.0, False))):
        for k in range(2):
            ph[k]["k0"] = wl["phases"][k]["k0"] * scale
            s.set_phase(k, ph[k])
        orc.step(g, ph, orc.StepOpts(tau=tau, passes=3), fo)
        st, _ = s.advance(o, report=report)
        assert st == 0
    assert rel_err(s.get_field("T1").cpu().numpy(), fo["T1"]) < 1e-12


@pytest.mark.parametrize("precision,whole", [("fp64", 0), ("fp32", 0), ("fp64", 1)])
def test_two_contexts_interleave_pipelined_steps(precision, whole):
    """Two contexts on the same stream take turns stepping without reports,
    so each has a pipelined step pending while the other enqueues and
    verifies its own.  Each context folds into its own pinned result blocks
    with its own sequence numbers: both runs must match their own oracle
    runs (grids of different sizes, so their schedules differ)."""
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    steps = 7
    runs = []
    for n in (160, 128):
        wl = W.levelset2d(n)
        tau, _ = oracle_dt(orc, wl)
        fo, _ = run_oracle(orc, wl, tau, steps)
        runs.append((make_solver(wl, precision), StepOpts(dt=tau, passes=3, whole_step=whole), fo))
    for s, o, _ in runs:
        assert s.advance(o)[0] == 0  # a reported first step each
    for _ in range(steps - 1):
        for s, o, _ in runs:
            assert s.advance(o, report=False)[0] == 0
    tol = 1e-12 if precision == "fp64" else 1e-5
    for s, _, fo in runs:
        assert s.finish() == 0
        _compare(fo, {k: s.get_field(k).cpu().numpy() for k in FIELDS_T}, FIELDS_T, tol)


def test_next_step_start_is_redone_after_changes():
    """The last launch of an FP64 step relaxes the next step's state and
    builds its first coefficients ahead of time.  Changing a field, the
    phases or alpha_eps between steps must discard that: each case is
    checked against the oracle doing the same."""
    import torch
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(160)
    tau, _ = oracle_dt(orc, wl)
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    fo = {k: v.copy() for k, v in wl["fields"].items()}
    s = make_solver(wl)
    ph = [dict(p) for p in wl["phases"]]
    for step in range(6):
        eps = 1e-10
        if step == 2:  # new temperatures
            for k in ("T1", "T2"):
                fo[k] = np.ascontiguousarray(fo["T1"] * 1.02)
                s.set_field(k, torch.from_numpy(fo[k].copy()))
        if step == 3:  # new conductivity
            ph[0]["k0"] *= 1.5
            s.set_phase(0, ph[0])
        if step == 4:
            eps = 1e-3
        orc.step(g, ph, orc.StepOpts(tau=tau, passes=3, alpha_eps=eps), fo)
        st, rep = s.advance(StepOpts(dt=tau, passes=3, alpha_eps=eps))
        assert st == 0
        assert rel_err(s.get_field("T1").cpu().numpy(), fo["T1"]) < 1e-12, step
        assert rel_err(s.get_field("alpha2").cpu().numpy(), fo["alpha2"]) < 1e-12, step


def test_paper_order_and_harmonic_faces():
    from oracle import oracle as orc
    wl = W.levelset2d(48)
    tau, _ = oracle_dt(orc, wl)
    tau *= 0.05  # tau*lambda = 20: the printed order is still accurate here
    for order, face in ((1, 0), (2, 1), (0, 1)):
        fo, ro = run_oracle(orc, wl, tau, 1, order=order, face_mean=face)
        fg, rg, _ = run_gpu(wl, tau, 1, frozen=_frozen(ro), order=order, face_mean=face)
        _compare(fo, fg, ("T1",), 1e-12)


def test_cycle_mode_reaches_backward_euler():
    """Cycle mode on heat1d agrees with the oracle's cycle mode and both with
    the direct tridiagonal BE solve."""
    from oracle import oracle as orc
    from scipy.linalg import solve_banded
    wl = W.heat1d()
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 1, passes=1, cycle_mode=1, cycle_tol=1e-14)
    fg, rg, _ = run_gpu(wl, tau, 1, passes=1, frozen=_frozen(ro), cycle_mode=1, cycle_tol=1e-14)
    assert rg[0]["residual"][0] < 1e-14
    g = orc.make_grid(wl["n"], wl["h"], wl["bc"])
    f = {k: v.copy() for k, v in wl["fields"].items()}
    orc.relax(g, wl["phases"], f["alpha2"], f["m1"], f["m2"], f["T1"], f["T2"])
    Lam = orc.cell_conductivity(g, wl["phases"], f["alpha2"], f["T1"]).ravel()
    Cap = orc.heat_capacity(g, wl["phases"], f["alpha2"], f["m1"], f["m2"], f["T1"]).ravel()
    Lf = 0.5 * (Lam[1:] + Lam[:-1]) / wl["h"][0] ** 2
    diag = Cap.copy()
    diag[:-1] += tau * Lf
    diag[1:] += tau * Lf
    ab = np.vstack([np.concatenate([[0.0], -tau * Lf]), diag, np.concatenate([-tau * Lf, [0.0]])])
    Tbe = solve_banded((1, 1), ab, Cap * f["T1"].ravel())
    assert rel_err(fg["T1"].ravel(), Tbe) < 1e-13
    assert rel_err(fg["T1"], fo["T1"]) < 1e-13


@pytest.mark.parametrize("sources,shape", [(True, (48, 48)), (False, (48, 48)), (False, (70, 33)),
                                           (True, (150, 130)), (False, (133, 140))])
def test_relaxation_unequal_pinf_and_sources(sources, shape):
    """Stiffened-gas phases (p_inf 6e8/0, Sec. 5 constants) out of thermal
    equilibrium, with and without heat sources: relaxation, C_eff, the alpha2
    update and the source term against the oracle.  Without sources the 2D
    relaxation runs fused with the first pass's coefficients."""
    from oracle import oracle as orc
    nx, ny = shape
    n = nx
    rng = np.random.default_rng(11)
    ph = [dict(gamma=4.4, pinf=6e8, cv=1606.0, q=0.0, k0=0.6, T0=300.0, npow=1.0, mu=0.0),
          dict(gamma=1.4, pinf=0.0, cv=714.0, q=0.0, k0=0.03, T0=300.0, npow=1.0, mu=0.0)]
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    a1 = 0.5 * (1 - np.tanh((x[None, :] - 0.5 - 0.1 * np.sin(2 * np.pi * y[:, None])) / (2.0 / nx)))
    a2 = 1 - a1
    rho1 = (1e9 + 6e8) / (3.4 * 1606.0 * 293.0)
    rho2 = 1e5 / (0.4 * 714.0 * 293.0)
    T1 = 293.0 + 20 * rng.random((ny, nx))
    T2 = 293.0 + 20 * rng.random((ny, nx))
    s1 = 1e3 * rng.random((1, ny, nx))
    s2 = 1e2 * rng.random((1, ny, nx))
    fields = dict(alpha2=a2.reshape(1, ny, nx), m1=(a1 * rho1).reshape(1, ny, nx),
                  m2=(a2 * rho2).reshape(1, ny, nx), T1=T1.reshape(1, ny, nx), T2=T2.reshape(1, ny, nx))
    if sources:
        fields.update(src1=s1, src2=s2)
    fields = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in fields.items()}
    wl = dict(n=(nx, ny, 1), h=(1e-3, 1e-3, 1.0), bc=(0, 1, 0), phases=ph, fields=fields, dt_factor=50.0,
              passes=3, viscous=False)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, frozen=_frozen(ro))
    _compare(fo, fg, FIELDS_T, 1e-12)


def test_picard_tolerance_and_noconv():
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts, E_NOCONV
    wl = W.levelset2d(32)
    tau, _ = oracle_dt(orc, wl)
    tau *= 0.1
    fo, ro = run_oracle(orc, wl, tau, 1, passes=40, picard_tol=1e-10)
    s = make_solver(wl)
    st, rep = s.advance(StepOpts(dt=tau, passes=40, picard_tol=1e-10))
    assert st == 0 and rep["converged"]
    assert rep["passes_run"] == ro[0]["passes_run"]
    assert rel_err(s.get_field("T1").cpu().numpy(), fo["T1"]) < 1e-12
    s2 = make_solver(wl)
    st, rep = s2.advance(StepOpts(dt=tau, passes=2, picard_tol=1e-15))
    assert st == E_NOCONV and not rep["converged"] and rep["passes_run"] == 2


def test_numeric_and_argument_errors():
    import torch
    from paper_2106_00282_amd.tlim import StepOpts, E_NUMERIC, E_ARG, TlimError
    wl = W.levelset2d(24)
    s = make_solver(wl)
    T = torch.from_numpy(wl["fields"]["T1"].copy())
    T[0, 3, 5] = float("nan")
    s.set_field("T1", T)
    s.set_field("T2", T)
    st, rep = s.advance(StepOpts(dt=1e-6))
    assert st == E_NUMERIC and rep["bad_cells"] >= 1
    with pytest.raises(TlimError) as ei:
        s.advance(StepOpts(dt=-1.0))
    assert ei.value.status == E_ARG
    with pytest.raises(TlimError):
        s.advance(StepOpts(dt=1e-6, passes=0))


def test_get_set_roundtrip_and_spectral_bound():
    import torch
    from oracle import oracle as orc
    wl = W.levelset2d(40)
    s = make_solver(wl)
    for k, v in wl["fields"].items():
        assert np.array_equal(s.get_field(k).cpu().numpy(), v)
    _, lam = oracle_dt(orc, wl)
    assert s.spectral_bound() == pytest.approx(lam, rel=1e-14)
    # the bound did not change the state
    assert np.array_equal(s.get_field("T1").cpu().numpy(), wl["fields"]["T1"])


def test_float32_field_buffers():
    """tlim_set_field / tlim_get_field with float32 buffers: the state keeps
    float64, widened exactly on the way in and rounded to nearest on the way
    out; a step from float32 inputs equals the step from the same values
    given in float64."""
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d(64)
    s = make_solver(wl)
    T32 = torch.from_numpy(wl["fields"]["T1"]).to(torch.float32)
    s.set_field("T1", T32)
    s.set_field("T2", T32)
    got = s.get_field("T1").cpu()
    assert torch.equal(got, T32.to(torch.float64))
    assert torch.equal(s.get_field("T2", dtype=torch.float32).cpu(), T32)
    full = torch.from_numpy(wl["fields"]["alpha2"])
    assert torch.equal(s.get_field("alpha2", dtype=torch.float32).cpu(), full.to(torch.float32))
    r = make_solver(wl)
    r.set_field("T1", T32.to(torch.float64))
    r.set_field("T2", T32.to(torch.float64))
    o = StepOpts(dt=1e-5, passes=2)
    assert s.advance(o)[0] == 0 and r.advance(o)[0] == 0
    assert torch.equal(s.get_field("T1"), r.get_field("T1"))


def test_whole_step_barrier_timeout_loses_the_state(monkeypatch):
    """A grid-barrier wait of the whole-step kernel that runs out (forced
    from the host: a spin limit of 0 polls, every kernel still exits) makes
    the step return TLIM_E_HIP and marks alpha2, T1 and T2 as not set, in
    the synchronous path and in the pipelined one; setting the fields again
    makes the context usable."""
    from paper_2106_00282_amd.tlim import E_HIP, E_STATE, StepOpts, TlimError
    wl = W.levelset2d(256)
    tau = wl["dt_factor"] * 2.0 / make_solver(wl).spectral_bound()
    monkeypatch.setenv("TLIM_STEP2D_SPIN_LIMIT", "0")
    sync, piped = make_solver(wl), make_solver(wl)
    monkeypatch.delenv("TLIM_STEP2D_SPIN_LIMIT")
    o = StepOpts(dt=tau, passes=3, whole_step=1)
    lost = 0
    for _ in range(3):
        try:
            sync.advance(o)
        except TlimError as e:
            assert e.status == E_HIP and "time-out" in str(e)
            lost += 1
            break
    assert lost == 1
    with pytest.raises(TlimError) as ei:
        sync.get_field("T1")
    assert ei.value.status == E_STATE
    with pytest.raises(TlimError) as ei:
        sync.advance(o)
    assert ei.value.status == E_STATE
    sync.set_workload(wl)
    # the pipelined path: the time-out is found by the call that verifies
    st = 0
    for _ in range(3):
        st = piped.advance_raw(o.c())
        if st != 0:
            break
    if st == 0:
        st = piped.finish()
    assert st == E_HIP
    with pytest.raises(TlimError):
        piped.get_field("alpha2")
    piped.set_workload(wl)
    # usable again (the spin limit is read per context: these still have 0,
    # so take the launch-per-block path)
    for s in (sync, piped):
        st, rep = s.advance(StepOpts(dt=tau, passes=3, whole_step=2))
        assert st == 0 and rep["bad_cells"] == 0


def test_single_cell_and_two_cell_periodic():
    from oracle import oracle as orc
    for n in ((1, 1, 1), (2, 1, 1), (2, 2, 2)):
        wl = W.levelset2d(8)
        N = n[0] * n[1] * n[2]
        rng = np.random.default_rng(N)
        for k in wl["fields"]:
            wl["fields"][k] = np.ascontiguousarray(wl["fields"][k].ravel()[:N].reshape(n[2], n[1], n[0]))
        wl["fields"]["T1"] = np.ascontiguousarray(1 + rng.random((n[2], n[1], n[0])))
        wl["fields"]["T2"] = wl["fields"]["T1"].copy()
        wl["n"] = n
        wl["h"] = tuple(1.0 / x if x > 1 else 1.0 for x in n)
        tau = 1e-3
        fo, ro = run_oracle(orc, wl, tau, 1)
        fg, rg, _ = run_gpu(wl, tau, 1, frozen=_frozen(ro))
        _compare(fo, fg, ("T1",), 1e-12)


# ------------------------------------------------------------------ FP32 form

def test_levelset2d_fp32_full_size():
    """FP32 sweeps, FP64 state and sums: per-field error against the FP64
    oracle at the benchmark workload (10 steps)."""
    from oracle import oracle as orc
    wl = W.levelset2d(1024)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 10)
    fg, rg, _ = run_gpu(wl, tau, 10, precision="fp32", frozen=_frozen(ro))
    errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
    print("fp32 per-field relative error vs FP64 oracle:", errs)
    assert errs["T1"] <= 1e-5 and errs["alpha2"] <= 1e-12
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-12


@pytest.mark.parametrize("shape,bc", [((100, 76), "periodic"), ((3, 130), "periodic"),
                                      ((130, 47), "adiabatic"), ((64, 64), "adiabatic"),
                                      ((200, 131), "adiabatic"), ((150, 260), "periodic")])
def test_levelset2d_fp32_ragged(shape, bc):
    """FP32 form on grids with ragged tiles and on adiabatic walls: the
    blocked float stages and the double final stage fused into the last
    launch, against the FP64 oracle (2 steps x 3 passes)."""
    from oracle import oracle as orc
    nx, ny = shape
    ng = max(128, nx, ny)
    wl = W.levelset2d(ng)
    for k in wl["fields"]:
        wl["fields"][k] = np.ascontiguousarray(wl["fields"][k][:, :ny, :nx])
    wl["n"] = (nx, ny, 1)
    wl["h"] = (1.0 / ng, 1.0 / ng, 1.0)
    if bc == "adiabatic":
        wl["bc"] = (W.ADIABATIC, W.ADIABATIC, W.PERIODIC)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, precision="fp32", frozen=_frozen(ro))
    errs = {k: rel_err(fg[k], fo[k]) for k in FIELDS_T}
    print("fp32 ragged per-field error:", shape, bc, errs)
    assert errs["T1"] <= 1e-5 and errs["T2"] <= 1e-5
    for r in rg:
        assert abs(r["energy_after"] / r["energy_before"] - 1) < 1e-12


def test_bubbles3d_fp32_with_viscous():
    from oracle import oracle as orc
    wl = W.bubbles3d(48)
    tau, _ = oracle_dt(orc, wl)
    fo, ro = run_oracle(orc, wl, tau, 2)
    fg, rg, _ = run_gpu(wl, tau, 2, precision="fp32", frozen=_frozen(ro))
    errs = {k: rel_err(fg[k], fo[k]) for k in ("T1", "u", "v", "w")}
    print("fp32 bubbles per-field error:", errs)
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)


# ------------------------------------------------------------------- adjoint

def _adjoint_setup(n=48, steps=3):
    from oracle import oracle as orc
    wl = W.levelset2d(n)
    tau, _ = oracle_dt(orc, wl)
    return orc, wl, tau, steps


def test_adjoint_vs_oracle_adjoint():
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    orc, wl, tau, steps = _adjoint_setup()
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    TN = s.get_field("T1").cpu().numpy()
    rng = np.random.default_rng(12)
    Tstar = wl["fields"]["T1"] * (1 + 0.05 * rng.standard_normal(TN.shape))
    dT0, dk0 = s.adjoint(opts, steps, 1, ckpt, lam, torch.from_numpy(TN - Tstar))
    f = wl["fields"]
    oopts = orc.StepOpts(tau=tau, passes=3)
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"], oopts, steps,
                                       np.array(lam), f["alpha2"], f["m1"], f["m2"], f["T1"], TN - Tstar)
    assert rel_err(TN, oTN) < 1e-12
    assert rel_err(dT0.cpu().numpy(), odT0) < 1e-12
    for k in range(2):
        assert dk0[k] == pytest.approx(odk0[k], rel=1e-12)
    # checkpoints every 2 steps give the same gradient
    s2 = make_solver(wl)
    ck2, lam2 = s2.forward_checkpointed(opts, steps, 2)
    d2, k2 = s2.adjoint(opts, steps, 2, ck2, lam2, torch.from_numpy(TN - Tstar))
    assert rel_err(d2.cpu().numpy(), dT0.cpu().numpy()) < 1e-13


@pytest.mark.parametrize("n", [140, 129])
def test_adjoint_wide_grids_vs_oracle_adjoint(n):
    """The adjoint on grids of 16-wave tiles with ragged last tiles (its
    recompute keeps the stages of the blocked forward kernel), against the
    oracle's adjoint."""
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    orc, wl, tau, steps = _adjoint_setup(n=n, steps=2)
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    TN = s.get_field("T1").cpu().numpy()
    g = TN - TN.mean()
    dT0, dk0 = s.adjoint(opts, steps, 1, ckpt, lam, torch.from_numpy(g))
    f = wl["fields"]
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"],
                                       orc.StepOpts(tau=tau, passes=3), steps, np.array(lam), f["alpha2"], f["m1"],
                                       f["m2"], f["T1"], g)
    assert rel_err(TN, oTN) < 1e-12
    assert rel_err(dT0.cpu().numpy(), odT0) < 1e-12
    for k in range(2):
        assert dk0[k] == pytest.approx(odk0[k], rel=1e-10)
    s.close()


def test_adjoint_in_fp32_context():
    """FP32 forward run (checkpoint at T^0 only): the adjoint recomputes and
    reverses in FP64, so with the run's schedule it equals the FP64 oracle
    adjoint from the same T^0."""
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    orc, wl, tau, steps = _adjoint_setup(n=64, steps=3)
    s = make_solver(wl, "fp32")
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, steps)
    TN32 = s.get_field("T1").cpu().numpy()
    rng = np.random.default_rng(13)
    g = 0.05 * rng.standard_normal(TN32.shape)
    dT0, dk0 = s.adjoint(opts, steps, steps, ckpt, lam, torch.from_numpy(g))
    f = wl["fields"]
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"],
                                       orc.StepOpts(tau=tau, passes=3), steps, np.array(lam), f["alpha2"], f["m1"],
                                       f["m2"], f["T1"], g)
    assert rel_err(TN32, oTN) < 1e-5
    assert rel_err(dT0.cpu().numpy(), odT0) < 1e-11
    for k in range(2):
        assert dk0[k] == pytest.approx(odk0[k], rel=1e-10)


@pytest.mark.parametrize("shape,steps,every", [((40, 40, 1), 5, 2), ((40, 36, 20), 4, 3), ((70, 24, 12), 3, 2)])
def test_adjoint_keeping_the_interval_equals_one_step_blocks(shape, steps, every):
    """The workspace that keeps every step of a checkpoint interval (each
    interval recomputed once) gives the same gradient, bit for bit, as the
    one that keeps one step (earlier steps of the interval recomputed for
    each later one), with a ragged last interval; and the oracle's."""
    import torch
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    if shape[2] == 1:
        wl = W.levelset2d(shape[0])
    else:
        wl = W.bubbles3d(shape[0], shape=shape)
        wl["viscous"] = False
        for k in ("u", "v", "w"):
            wl["fields"].pop(k)
    tau, _ = oracle_dt(orc, wl)
    print(f"case adjoint kept interval {wl['n']} steps={steps} every={every}", flush=True)
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, every)
    TN = s.get_field("T1").cpu().numpy()
    # L = |T^N - mean|^2 / 2: conduction lowers it everywhere, so the terms
    # of dL/dk0 share their sign and the sum keeps the fields' agreement
    g = torch.from_numpy(TN - TN.mean())
    d1, k1 = s.adjoint(opts, steps, every, ckpt, lam, g, keep_interval=False)
    n1 = s._adj_ws.numel()
    d1 = d1.cpu().numpy()
    s._adj_ws = None
    dk, kk = s.adjoint(opts, steps, every, ckpt, lam, g, keep_interval=True)
    assert s._adj_ws.numel() > n1
    assert np.array_equal(dk.cpu().numpy(), d1)
    assert kk == k1
    f = wl["fields"]
    odT0, odk0, _ = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"],
                                     orc.StepOpts(tau=tau, passes=3), steps, np.array(lam), f["alpha2"], f["m1"],
                                     f["m2"], f["T1"], g.numpy())
    assert rel_err(d1, odT0) < 1e-12
    for k in range(2):
        assert k1[k] == pytest.approx(odk0[k], rel=1e-11)
    s.close()


@pytest.mark.parametrize("case", ["harmonic2d", "grid3d", "adiabatic2d"])
def test_adjoint_other_paths_vs_oracle(case):
    """The adjoint on grids and face means outside the blocked 2D path
    (harmonic face mean, 3D grid) and on an adiabatic 2D grid, against the
    oracle's adjoint."""
    import torch
    from oracle import oracle as orc
    from paper_2106_00282_amd.tlim import StepOpts
    face = 1 if case == "harmonic2d" else 0
    if case == "grid3d":
        wl = W.bubbles3d(20)
        wl["viscous"] = False
        for k in ("u", "v", "w"):
            wl["fields"].pop(k)
    else:
        wl = W.levelset2d(40)
        if case == "adiabatic2d":
            wl["bc"] = (1, 1, 0)
    tau, _ = oracle_dt(orc, wl)
    steps = 2
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3, face_mean=face)
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    TN = s.get_field("T1").cpu().numpy()
    rng = np.random.default_rng(14)
    w = rng.standard_normal(TN.shape)
    dT0, dk0 = s.adjoint(opts, steps, 1, ckpt, lam, torch.from_numpy(w))
    f = wl["fields"]
    oopts = orc.StepOpts(tau=tau, passes=3, face_mean=face)
    odT0, odk0, oTN = orc.heat_adjoint(orc.make_grid(wl["n"], wl["h"], wl["bc"]), wl["phases"], oopts, steps,
                                       np.array(lam), f["alpha2"], f["m1"], f["m2"], f["T1"], w)
    assert rel_err(TN, oTN) < 1e-12
    assert rel_err(dT0.cpu().numpy(), odT0) < 1e-12
    # dL/dk0 is a sum over every cell and pass whose terms carry the ~1e-12
    # relative agreement of the fields; with a random loss weight the terms
    # cancel (their net is ~30x smaller than their size here), so the sum is
    # held at 1e-10
    for k in range(2):
        assert dk0[k] == pytest.approx(odk0[k], rel=1e-10)


def test_autograd_function_vs_central_fd():
    """torch.autograd through ParabolicRun against central differences of the
    GPU forward (frozen schedule) on 16 cells and both k0."""
    import torch
    from paper_2106_00282_amd.tlim import ParabolicRun, StepOpts
    orc, wl, tau, steps = _adjoint_setup(40, 3)
    s = make_solver(wl)
    opts = StepOpts(dt=tau, passes=3)
    dev = s.device
    T0 = torch.from_numpy(wl["fields"]["T1"].copy()).to(dev).requires_grad_(True)
    k0 = torch.tensor([wl["phases"][0]["k0"], wl["phases"][1]["k0"]], dtype=torch.float64, device=dev,
                      requires_grad=True)
    rng = np.random.default_rng(13)
    Tstar = torch.from_numpy(wl["fields"]["T1"] * (1 + 0.05 * rng.standard_normal(wl["fields"]["T1"].shape))).to(dev)
    TN = ParabolicRun.apply(T0, k0, s, opts, steps, 1, wl["phases"])
    loss = 0.5 * ((TN - Tstar) ** 2).sum()
    loss.backward()
    lam = None

    def fwd_loss(T0v, k0v):
        nonlocal lam
        ph = [dict(p) for p in wl["phases"]]
        for k in range(2):
            ph[k]["k0"] = float(k0v[k])
            s.set_phase(k, ph[k])
        s.set_field("T1", T0v)
        s.set_field("T2", T0v)
        for n in range(steps):
            o = StepOpts(dt=tau, passes=3, frozen_lambda=lam[3 * n:3 * n + 3])
            st, _ = s.advance(o)
            assert st == 0
        r = s.get_field("T1") - Tstar
        return 0.5 * float((r * r).sum())

    # the schedule of the recorded forward run
    s2 = make_solver(wl)
    _, lam = s2.forward_checkpointed(opts, steps, 1)
    cells = rng.choice(T0.numel(), size=16, replace=False)
    base = T0.detach().clone()
    for c in cells:
        # step 1e-3: truncation ~2e-7 relative.  The forward carries a
        # rounding floor of ~tau*lambda*eps per pass, which a smaller step
        # turns into FD noise of 1e-6 (1e-4) to 4e-5 (1e-5)
        hstep = 1e-3 * float(base.view(-1)[c])
        Tp, Tm = base.clone(), base.clone()
        Tp.view(-1)[c] += hstep
        Tm.view(-1)[c] -= hstep
        fd = (fwd_loss(Tp, k0.detach()) - fwd_loss(Tm, k0.detach())) / (2 * hstep)
        g = float(T0.grad.view(-1)[c])
        assert g == pytest.approx(fd, rel=1e-6, abs=1e-9 * float(T0.grad.abs().max()))
    for k in range(2):
        hstep = 1e-4 * float(k0[k])
        kp, km = k0.detach().clone(), k0.detach().clone()
        kp[k] += hstep
        km[k] -= hstep
        fd = (fwd_loss(base, kp) - fwd_loss(base, km)) / (2 * hstep)
        assert float(k0.grad[k]) == pytest.approx(fd, rel=1e-6)


# ------------------------------------------------ adjoint at the full sizes

def _frozen_loss(s, wl, tau, lam, steps, T0, k0, Tstar):
    """L = 1/2 sum (T^N - T*)^2 of the GPU forward from (T0, k0) with the
    recorded schedule frozen."""
    from paper_2106_00282_amd.tlim import StepOpts
    ph = [dict(p) for p in wl["phases"]]
    for k in range(2):
        ph[k]["k0"] = float(k0[k])
        s.set_phase(k, ph[k])
    s.set_field("T1", T0)
    s.set_field("T2", T0)
    for n in range(steps):
        st, _ = s.advance(StepOpts(dt=tau, passes=3, frozen_lambda=lam[3 * n:3 * n + 3]), report=False)
        assert st == 0
    r = s.get_field("T1") - Tstar
    return 0.5 * float((r * r).sum())


def _target(wl, tau, steps, precision="fp64"):
    """T^N of the run with both k0 scaled by the workload's target factor."""
    from paper_2106_00282_amd.tlim import StepOpts
    wt = dict(wl)
    wt["phases"] = [dict(p, k0=p["k0"] * wl.get("target_k0_scale", 1.1)) for p in wl["phases"]]
    st = make_solver(wt, precision)
    for _ in range(steps):
        assert st.advance(StepOpts(dt=tau, passes=3), report=False)[0] == 0
    assert st.finish() == 0
    out = st.get_field("T1")
    st.close()
    return out


def test_adjoint_full_size_2048_fd():
    """The 2048^2, 20-step adjoint workload (checkpoint every step): the
    gradient w.r.t. the 16 probe cells of T^0 and both k0 against central
    differences of the frozen-schedule GPU forward."""
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.levelset2d_adjoint(2048, 20)
    steps = wl["steps"]
    s = make_solver(wl)
    tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
    Tstar = _target(wl, tau, steps)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 1)
    TN = s.get_field("T1")
    dT0, dk0 = s.adjoint(opts, steps, 1, ckpt, lam, TN - Tstar)
    base = torch.from_numpy(wl["fields"]["T1"].copy()).to(s.device)
    k0 = [p["k0"] for p in wl["phases"]]
    gmax = float(dT0.abs().max())

    def fd_cell(c, h):
        Tp, Tm = base.clone(), base.clone()
        Tp.view(-1)[c] += h
        Tm.view(-1)[c] -= h
        return (_frozen_loss(s, wl, tau, lam, steps, Tp, k0, Tstar) -
                _frozen_loss(s, wl, tau, lam, steps, Tm, k0, Tstar)) / (2 * h)

    def fd_k0(k, h):
        kp, km = list(k0), list(k0)
        kp[k] += h
        km[k] -= h
        return (_frozen_loss(s, wl, tau, lam, steps, base, kp, Tstar) -
                _frozen_loss(s, wl, tau, lam, steps, base, km, Tstar)) / (2 * h)

    # central differences at h and h/2, extrapolated (Richardson): the O(h^2)
    # truncation of the 20-step nonlinear forward is ~1e-6 at h = 1e-3
    for c in wl["fd_cells"]:
        h = 1e-3 * float(base.view(-1)[int(c)])
        fd = (4 * fd_cell(int(c), h / 2) - fd_cell(int(c), h)) / 3
        assert float(dT0.view(-1)[int(c)]) == pytest.approx(fd, rel=1e-6, abs=1e-9 * gmax), c
    for k in range(2):
        h = 1e-3 * k0[k]
        fd = (4 * fd_k0(k, h / 2) - fd_k0(k, h)) / 3
        assert dk0[k] == pytest.approx(fd, rel=1e-6), k


def test_adjoint_full_size_512cube_directional():
    """The 512^3 interface workload, 10 steps with checkpoints every 2 steps
    (about 140 GB of device memory with the stage storage): the adjoint's
    directional derivative along a random (T^0, k0) direction against a
    central difference of the frozen-schedule forward."""
    import torch
    from paper_2106_00282_amd.tlim import StepOpts
    wl = W.interface3d(512, steps=10)
    steps = wl["steps"]
    s = make_solver(wl)
    tau = wl["dt_factor"] * 2.0 / s.spectral_bound()
    Tstar = _target(wl, tau, steps)
    opts = StepOpts(dt=tau, passes=3)
    ckpt, lam = s.forward_checkpointed(opts, steps, 2)
    TN = s.get_field("T1")
    dT0, dk0 = s.adjoint(opts, steps, 2, ckpt, lam, TN - Tstar)
    del ckpt
    gen = torch.Generator(device=s.device).manual_seed(5)
    base = torch.from_numpy(wl["fields"]["T1"]).to(s.device)
    dT = 1e-3 * base * torch.rand(base.shape, generator=gen, device=s.device, dtype=torch.float64)
    k0 = [p["k0"] for p in wl["phases"]]
    dk = [0.3 * k0[0], -0.2 * k0[1]]
    dadj = float((dT0 * dT).sum()) + dk0[0] * dk[0] + dk0[1] * dk[1]

    def fd(eps):
        Lp = _frozen_loss(s, wl, tau, lam, steps, base + eps * dT, [k0[i] + eps * dk[i] for i in range(2)], Tstar)
        Lm = _frozen_loss(s, wl, tau, lam, steps, base - eps * dT, [k0[i] - eps * dk[i] for i in range(2)], Tstar)
        return (Lp - Lm) / (2 * eps)

    dfd = (4 * fd(5e-4) - fd(1e-3)) / 3  # Richardson-extrapolated central difference
    assert dadj == pytest.approx(dfd, rel=1e-6)
