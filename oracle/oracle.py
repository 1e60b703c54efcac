"""ctypes wrapper of the FP64 CPU oracle (``tlim_oracle.c``).

Test infrastructure only: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.

Arrays are numpy float64, C-contiguous, shaped (nz, ny, nx) -- x fastest --
exactly as the C code indexes them.  Function docstrings name the passage of
arXiv 2106.00282 each C routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tlim_oracle.c")
LIB = os.path.join(HERE, "libtlim_oracle.so")

PERIODIC, ADIABATIC = 0, 1
ORDER_INTERLEAVED, ORDER_PAPER, ORDER_ASCENDING = 0, 1, 2
FACE_ARITH, FACE_HARMONIC = 0, 1
LAW_POWER, LAW_SPITZER = 0, 1
MAX_PASSES = 64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Grid(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 3)]


class Phase(C.Structure):
    _fields_ = ([(k, C.c_double) for k in ("gamma", "pinf", "cv", "q", "k0", "T0", "npow", "mu")] +
                [("law", C.c_int32)] + [(k, C.c_double) for k in ("sh_D", "sh_LD", "sh_dB")])


class Opts(C.Structure):
    _fields_ = [("tau", C.c_double), ("passes", C.c_int32), ("picard_tol", C.c_double),
                ("order", C.c_int32), ("face_mean", C.c_int32), ("cycle_mode", C.c_int32),
                ("cycle_tol", C.c_double), ("max_cycles", C.c_int32), ("alpha_eps", C.c_double),
                ("do_viscous", C.c_int32), ("visc_heating", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("passes_run", C.c_int32), ("converged", C.c_int32),
                ("P", C.c_int32 * MAX_PASSES), ("lambda_G", C.c_double * MAX_PASSES),
                ("err", C.c_double * MAX_PASSES), ("cycles", C.c_int32 * MAX_PASSES),
                ("residual", C.c_double * MAX_PASSES), ("visc_P", C.c_int32 * 3),
                ("visc_lambda_G", C.c_double * 3), ("energy_before", C.c_double),
                ("energy_after", C.c_double)]


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        L.orc_lim_P.restype = C.c_int32
        L.orc_lim_P.argtypes = [C.c_double, C.c_double]
        L.orc_lim_params.argtypes = [C.c_int32, C.c_double, C.c_int32, _dp]
        L.orc_cycle_params.argtypes = [C.c_int32, C.c_double, _dp]
        L.orc_cell_conductivity.argtypes = [C.POINTER(Grid), C.POINTER(Phase), _dp, _dp, _dp, _dp, _dp]
        L.orc_heat_capacity.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_double,
                                        _dp, _dp, _dp, _dp, _dp]
        L.orc_gershgorin.restype = C.c_double
        L.orc_gershgorin.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_int32]
        L.orc_apply_A.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_int32, _dp, _dp]
        L.orc_lim_pass.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_int32, C.c_double,
                                   C.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.orc_relax.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_energy.restype = C.c_double
        L.orc_energy.argtypes = [C.POINTER(Grid), C.POINTER(Phase), _dp, _dp, _dp, _dp, _dp]
        L.orc_step.restype = C.c_int32
        L.orc_step.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.POINTER(Opts),
                               _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                               C.POINTER(Report)]
        L.orc_cycle_solve.restype = C.c_int32
        L.orc_cycle_solve.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_int32, C.c_double,
                                      C.c_double, C.c_int32, _dp, _dp, C.c_double, C.c_int32,
                                      _dp, _dp]
        L.orc_be_residual.restype = C.c_double
        L.orc_be_residual.argtypes = [C.POINTER(Grid), _dp, _dp, _dp, C.c_int32, C.c_double, _dp, _dp]
        L.orc_visc_heat.restype = None
        L.orc_visc_heat.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_double, C.c_int32, _dp, _dp, _dp, _dp,
                                    _dp, C.c_double, _dp, _dp, _dp]
        L.orc_visc_energy.restype = None
        L.orc_visc_energy.argtypes = [C.POINTER(Grid), C.c_int32, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_heat_adjoint.restype = C.c_int32
        L.orc_heat_adjoint.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.POINTER(Opts), C.c_int32,
                                       _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_hyperbolic.restype = C.c_int32
        L.orc_hyperbolic.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_double, C.c_int32] + [_dp] * 9
        L.orc_pressure_relax_cell.restype = None
        L.orc_pressure_relax_cell.argtypes = [C.POINTER(Phase), _dp]
        L.orc_hyperbolic_dt.restype = C.c_double
        L.orc_hyperbolic_dt.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_double] + [_dp] * 8
        _lib = L
    return _lib


def _p(a, n=None):
    """Pointer to a C-contiguous float64 array, checked to hold n values."""
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError("oracle arrays are C-contiguous float64 numpy arrays")
    if n is not None and a.size != n:
        raise ValueError(f"array has {a.size} values, the grid has {n}")
    return a.ctypes.data_as(_dp)


def _ncell(g) -> int:
    return int(g.n[0] * g.n[1] * g.n[2])


def make_grid(n, h=None, bc=None) -> Grid:
    """n = (nx, ny, nz); h defaults to 1/n per axis (unit box), bc to periodic."""
    n = tuple(int(x) for x in n) + (1,) * (3 - len(n))
    if h is None:
        h = tuple(1.0 / x if x > 1 else 1.0 for x in n)
    h = tuple(float(x) for x in h) + (1.0,) * (3 - len(h))
    bc = tuple(bc) if bc is not None else (PERIODIC,) * 3
    bc = bc + (PERIODIC,) * (3 - len(bc))
    g = Grid()
    for d in range(3):
        g.n[d], g.h[d], g.bc[d] = n[d], h[d], bc[d]
    return g


def make_phases(ph):
    arr = (Phase * 2)()
    for k in range(2):
        p = ph[k]
        for name in ("gamma", "pinf", "cv", "q", "k0", "T0", "npow", "mu"):
            setattr(arr[k], name, float(p.get(name, 0.0 if name not in ("gamma", "T0") else 1.0)))
        arr[k].law = int(p.get("law", LAW_POWER))
        for name in ("sh_D", "sh_LD", "sh_dB"):
            setattr(arr[k], name, float(p.get(name, 0.0)))
    return arr


@dataclass
class StepOpts:
    tau: float
    passes: int = 3
    picard_tol: float = 0.0
    order: int = ORDER_INTERLEAVED
    face_mean: int = FACE_ARITH
    cycle_mode: int = 0
    cycle_tol: float = 1e-14
    max_cycles: int = 200
    alpha_eps: float = 1e-10
    do_viscous: int = 0
    visc_heating: int = 0

    def c(self) -> Opts:
        o = Opts()
        for k in ("tau", "passes", "picard_tol", "order", "face_mean", "cycle_mode",
                  "cycle_tol", "max_cycles", "alpha_eps", "do_viscous", "visc_heating"):
            setattr(o, k, getattr(self, k))
        return o


# ---------------------------------------------------------------- building blocks

def lim_P(tau, lam):
    """P = ceil(pi/4 sqrt(tau lambda_max + 1)) (Sec. 3.2, eq. LIM)."""
    return int(lib().orc_lim_P(tau, lam))


def lim_params(P, lam, order=ORDER_INTERLEAVED):
    """b_1..b_{2P-1} of one LIM pass (Sec. 3.2, definition of a_m and beta_j)."""
    b = np.zeros(2 * P - 1)
    lib().orc_lim_params(P, lam, order, _p(b))
    return b


def cycle_params(s, lam):
    b = np.zeros(s)
    lib().orc_cycle_params(s, lam, _p(b))
    return b


def cell_conductivity(g, ph, alpha2, T, m1=None, m2=None):
    """Lambda = sum_k alpha_k lambda_k(rho, T) (Sec. 3.4.2, eq. qk_dis), rho = m1 + m2
    (needed only by the Spitzer-Harm law of Sec. 4.4)."""
    N = _ncell(g)
    out = np.empty_like(T)
    lib().orc_cell_conductivity(C.byref(g), make_phases(ph), _p(alpha2, N), _p(m1, N), _p(m2, N),
                                _p(T, N), _p(out, N))
    return out


def heat_capacity(g, ph, alpha2, m1, m2, T, eps=1e-10):
    N = _ncell(g)
    out = np.empty_like(T)
    lib().orc_heat_capacity(C.byref(g), make_phases(ph), eps, _p(alpha2, N), _p(m1, N), _p(m2, N), _p(T, N), _p(out, N))
    return out


def gershgorin(g, Lam, Cap, scale=(1.0, 1.0, 1.0), face_mean=FACE_ARITH):
    N = _ncell(g)
    s = np.asarray(scale, dtype=np.float64)
    return float(lib().orc_gershgorin(C.byref(g), _p(Lam, N), _p(Cap, N), _p(s), face_mean))


def apply_A(g, Lam, Cap, v, scale=(1.0, 1.0, 1.0), face_mean=FACE_ARITH):
    N = _ncell(g)
    s = np.asarray(scale, dtype=np.float64)
    y = np.empty_like(v)
    lib().orc_apply_A(C.byref(g), _p(Lam, N), _p(Cap, N), _p(s), face_mean, _p(v, N), _p(y, N))
    return y


def lim_pass(g, Lam, Cap, tau, b, rhs, v0, scale=(1.0, 1.0, 1.0), face_mean=FACE_ARITH,
             keep_stages=False):
    """One LIM pass, eqs. LIM and LIM_last (Sec. 3.2)."""
    N = _ncell(g)
    s = np.asarray(scale, dtype=np.float64)
    out = np.empty_like(rhs)
    b = np.ascontiguousarray(b, dtype=np.float64)
    st = np.empty((len(b),) + rhs.shape) if keep_stages else None
    lib().orc_lim_pass(C.byref(g), _p(Lam, N), _p(Cap, N), _p(s), face_mean, tau, len(b), _p(b),
                       _p(rhs, N), _p(v0, N), _p(out, N), _p(st) if st is not None else None)
    return (out, st) if keep_stages else out


def cycle_solve(g, Lam, Cap, tau, lam, s, rhs, v0, tol=1e-14, max_cycles=200,
                scale=(1.0, 1.0, 1.0), face_mean=FACE_ARITH):
    N = _ncell(g)
    sc = np.asarray(scale, dtype=np.float64)
    out = np.empty_like(rhs)
    hist = np.zeros(max(max_cycles, 1))
    nc = lib().orc_cycle_solve(C.byref(g), _p(Lam, N), _p(Cap, N), _p(sc), face_mean, tau, lam, s,
                               _p(rhs, N), _p(v0, N), tol, max_cycles, _p(out, N), _p(hist))
    return out, hist[:nc]


def be_residual(g, Lam, Cap, tau, rhs, v, scale=(1.0, 1.0, 1.0), face_mean=FACE_ARITH):
    N = _ncell(g)
    sc = np.asarray(scale, dtype=np.float64)
    return float(lib().orc_be_residual(C.byref(g), _p(Lam, N), _p(Cap, N), _p(sc), face_mean, tau, _p(rhs, N), _p(v, N)))


def relax(g, ph, alpha2, m1, m2, T1, T2, eps=1e-10):
    """Temperature relaxation in mixed cells, in place (Sec. 3.4.1)."""
    N = _ncell(g)
    lib().orc_relax(C.byref(g), make_phases(ph), eps, _p(alpha2, N), _p(m1, N), _p(m2, N), _p(T1, N), _p(T2, N))


def visc_heat(g, ph, alpha2, m1, m2, mu, scale, tau, uh, T1, T2, eps=1e-10, face_mean=FACE_ARITH):
    """Viscous heating of the phases by one velocity component, in place on
    T1, T2 (Sec. 3.2, phase internal energies); uh the predicted velocity."""
    N = _ncell(g)
    sc = np.asarray(scale, dtype=np.float64)
    lib().orc_visc_heat(C.byref(g), make_phases(ph), eps, face_mean, _p(alpha2, N), _p(m1, N), _p(m2, N), _p(mu, N),
                        _p(sc), tau, _p(uh, N), _p(T1, N), _p(T2, N))


def visc_energy(g, mu, scale, tau, uh, E, face_mean=FACE_ARITH):
    """Total-energy update of the viscous part by one velocity component, in
    place on E (Sec. 3.2); uh the predicted velocity."""
    N = _ncell(g)
    sc = np.asarray(scale, dtype=np.float64)
    lib().orc_visc_energy(C.byref(g), face_mean, _p(mu, N), _p(sc), tau, _p(uh, N), _p(E, N))


def energy(g, ph, alpha2, m1, m2, T1, T2):
    N = _ncell(g)
    return float(lib().orc_energy(C.byref(g), make_phases(ph), _p(alpha2, N), _p(m1, N), _p(m2, N), _p(T1, N), _p(T2, N)))


def _report(r: Report, passes: int):
    n = r.passes_run
    return dict(passes_run=n, converged=bool(r.converged), P=list(r.P[:n]),
                lambda_G=list(r.lambda_G[:n]), err=list(r.err[:n]), cycles=list(r.cycles[:n]),
                residual=list(r.residual[:n]), visc_P=list(r.visc_P), visc_lambda_G=list(r.visc_lambda_G),
                energy_before=r.energy_before, energy_after=r.energy_after)


def step(g, ph, opts: StepOpts, f: dict, frozen_lambda=None, frozen_visc=None):
    """One parabolic step (viscous, relaxation, Algorithm 1) on the fields of
    ``f`` in place; the total energy f["E"] is updated when present.
    Returns (status, report dict)."""
    N = _ncell(g)
    rep = Report()
    fl = None if frozen_lambda is None else np.ascontiguousarray(frozen_lambda, dtype=np.float64)
    fv = None if frozen_visc is None else np.ascontiguousarray(frozen_visc, dtype=np.float64)
    if fl is not None and fl.size < opts.passes:
        raise ValueError("frozen_lambda needs one value per pass")
    if fv is not None and fv.size < 3:
        raise ValueError("frozen_visc needs 3 values")
    st = lib().orc_step(C.byref(g), make_phases(ph), C.byref(opts.c()), _p(f["alpha2"], N), _p(f["m1"], N),
                        _p(f["m2"], N), _p(f["T1"], N), _p(f["T2"], N), _p(f.get("src1"), N), _p(f.get("src2"), N),
                        _p(f.get("u"), N), _p(f.get("v"), N), _p(f.get("w"), N), _p(f.get("E"), N),
                        _p(fl) if fl is not None else None, _p(fv) if fv is not None else None,
                        C.byref(rep))
    return int(st), _report(rep, opts.passes)


def heat_adjoint(g, ph, opts: StepOpts, nsteps, lamsched, alpha2, m1, m2, T0, dL_dTN):
    """Discrete adjoint of ``nsteps`` heat steps with a frozen schedule.
    Returns (dL/dT0, dL/dk0[2], T^N)."""
    N = _ncell(g)
    lamsched = np.ascontiguousarray(lamsched, dtype=np.float64).ravel()
    if lamsched.size < nsteps * opts.passes:
        raise ValueError("the schedule needs nsteps * passes values")
    dT0 = np.empty_like(T0)
    dk0 = np.zeros(2)
    TN = np.empty_like(T0)
    st = lib().orc_heat_adjoint(C.byref(g), make_phases(ph), C.byref(opts.c()), nsteps, _p(lamsched),
                                _p(alpha2, N), _p(m1, N), _p(m2, N), _p(T0, N), _p(dL_dTN, N), _p(dT0, N), _p(dk0), _p(TN, N))
    if st != 0:
        raise ValueError("oracle adjoint: unsupported configuration")
    return dT0, dk0, TN


# ------------------------------------------------------- hyperbolic part

def hyperbolic(g, ph, dt, f: dict, relax_pressure=True):
    """One Godunov-HLLC step of the hyperbolic part (Sec. 3.1, dimensional
    splitting) and the pressure relaxation (Sec. 3.3), in place on the fields
    of f (alpha2, m1, m2, T1, T2; u, v, w and E when present).  Returns 1 if a
    cell left 0 < alpha2 < 1 or lost a positive temperature."""
    N = _ncell(g)
    return int(lib().orc_hyperbolic(C.byref(g), make_phases(ph), dt, int(relax_pressure),
                                    *[_p(f.get(k), N) for k in ("alpha2", "m1", "m2", "T1", "T2",
                                                                 "u", "v", "w", "E")]))


def pressure_relax_cell(ph, q):
    """Pressure relaxation (Sec. 3.3) of one conservative state q[9]; returns
    the relaxed copy."""
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    lib().orc_pressure_relax_cell(make_phases(ph), _p(q, 9))
    return q


def hyperbolic_dt(g, ph, cfl, f: dict):
    N = _ncell(g)
    return float(lib().orc_hyperbolic_dt(C.byref(g), make_phases(ph), cfl,
                                         *[_p(f.get(k), N) for k in ("alpha2", "m1", "m2", "T1", "T2",
                                                                      "u", "v", "w")]))
