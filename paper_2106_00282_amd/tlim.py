"""Python binding of libtlim (C ABI in include/tlim.h).

Argument marshalling only: every step of the parabolic sub-step runs in the
library's HIP kernels.  PyTorch provides the device memory (the workspace
and the field tensors) and the stream.  There is no fallback: if the
library is missing or no HIP device is present, construction fails.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass, field as dc_field
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtlim.so")

OK, E_ARG, E_STATE, E_HIP, E_NOMEM, E_NOCONV, E_NUMERIC = range(7)
PERIODIC, ADIABATIC = 0, 1
FP64, FP32 = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1  # element type of a field buffer (tlim_set_field / tlim_get_field)
_DTYPES = {torch.float64: DTYPE_F64, torch.float32: DTYPE_F32}
ORDER_INTERLEAVED, ORDER_PAPER, ORDER_ASCENDING = 0, 1, 2
FACE_ARITH, FACE_HARMONIC = 0, 1
WHOLE_AUTO, WHOLE_ALWAYS, WHOLE_NEVER = 0, 1, 2
LAW_POWER, LAW_SPITZER = 0, 1  # conductivity laws (tlim_phase.law)
FIELDS = dict(alpha2=0, m1=1, m2=2, T1=3, T2=4, u=5, v=6, w=7, src1=8, src2=9, E=10)
MAX_PASSES = 64

EXPORTED = ("tlim_create", "tlim_destroy", "tlim_workspace_bytes", "tlim_bind_workspace",
            "tlim_set_phase", "tlim_set_field", "tlim_get_field", "tlim_clear_field", "tlim_spectral_bound",
            "tlim_advance_parabolic", "tlim_finish", "tlim_forward_checkpointed", "tlim_adjoint_workspace_bytes",
            "tlim_adjoint_workspace_bytes_kept",
            "tlim_adjoint_parabolic", "tlim_advance_hyperbolic", "tlim_hyperbolic_dt", "tlim_status_str",
            "tlim_last_error", "tlim_spectral_bound_noalloc")


class TlimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 3)]


class Phase(C.Structure):
    _fields_ = ([(k, C.c_double) for k in ("gamma", "pinf", "cv", "q", "k0", "T0", "npow", "mu")] +
                [("law", C.c_int32)] + [(k, C.c_double) for k in ("sh_D", "sh_LD", "sh_dB")])


class StepOptsC(C.Structure):
    _fields_ = [("dt", C.c_double), ("passes", C.c_int32), ("picard_tol", C.c_double),
                ("order", C.c_int32), ("face_mean", C.c_int32), ("cycle_mode", C.c_int32),
                ("cycle_tol", C.c_double), ("max_cycles", C.c_int32), ("alpha_eps", C.c_double),
                ("do_viscous", C.c_int32), ("frozen_lambda", C.POINTER(C.c_double)),
                ("frozen_visc", C.POINTER(C.c_double)), ("time_sweeps", C.c_int32),
                ("visc_heating", C.c_int32), ("whole_step", C.c_int32)]


class HypOptsC(C.Structure):
    _fields_ = [("dt", C.c_double), ("relax_pressure", C.c_int32)]


class HypReportC(C.Structure):
    _fields_ = [("bad_cells", C.c_double)]


class ReportC(C.Structure):
    _fields_ = [("passes_run", C.c_int32), ("converged", C.c_int32),
                ("P", C.c_int32 * MAX_PASSES), ("lambda_G", C.c_double * MAX_PASSES),
                ("err", C.c_double * MAX_PASSES), ("cycles", C.c_int32 * MAX_PASSES),
                ("residual", C.c_double * MAX_PASSES), ("visc_P", C.c_int32 * 3),
                ("visc_lambda_G", C.c_double * 3), ("energy_before", C.c_double),
                ("energy_after", C.c_double), ("sweeps", C.c_int64), ("sweep_launches", C.c_int64),
                ("sweep_ms", C.c_double), ("bad_cells", C.c_int64), ("predicted", C.c_int32),
                ("mispredicted", C.c_int32), ("pipelined_steps", C.c_int64), ("pipeline_redos", C.c_int64),
                ("timed_sweeps", C.c_int64), ("timed_launches", C.c_int64)]


_lib = None
# Contexts still open when the interpreter exits are closed by the atexit
# hook below, while the HIP runtime and torch are still fully alive, rather
# than by __del__ during module teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def load_library(path: str = LIB_PATH):
    """Load libtlim.so and declare its signatures (no device call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtlim.so not found at {path}: build it with "
                          f"`python -m paper_2106_00282_amd.build` (hipcc, gfx950)")
    L = C.CDLL(path)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.tlim_create.argtypes = [C.POINTER(Grid), C.c_int32, vp, C.POINTER(vp)]
    L.tlim_destroy.argtypes = [vp]
    L.tlim_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.tlim_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.tlim_set_phase.argtypes = [vp, C.c_int32, C.POINTER(Phase)]
    L.tlim_set_field.argtypes = [vp, C.c_int32, vp, C.c_int32]
    L.tlim_get_field.argtypes = [vp, C.c_int32, vp, C.c_int32]
    L.tlim_clear_field.argtypes = [vp, C.c_int32]
    L.tlim_spectral_bound.argtypes = [vp, C.c_int32, C.c_double, dp]
    L.tlim_advance_parabolic.argtypes = [vp, C.POINTER(StepOptsC), C.POINTER(ReportC)]
    L.tlim_finish.argtypes = [vp]
    L.tlim_forward_checkpointed.argtypes = [vp, C.POINTER(StepOptsC), C.c_int32, C.c_int32, vp, dp]
    L.tlim_adjoint_workspace_bytes.argtypes = [vp, C.POINTER(StepOptsC), C.c_int32, dp, C.POINTER(C.c_size_t)]
    L.tlim_adjoint_workspace_bytes_kept.argtypes = [vp, C.POINTER(StepOptsC), C.c_int32, C.c_int32, dp,
                                                    C.POINTER(C.c_size_t)]
    L.tlim_adjoint_parabolic.argtypes = [vp, C.POINTER(StepOptsC), C.c_int32, C.c_int32, vp, dp, vp, vp, dp, vp,
                               C.c_size_t]
    L.tlim_status_str.restype = C.c_char_p
    L.tlim_advance_hyperbolic.argtypes = [vp, C.POINTER(HypOptsC), C.POINTER(HypReportC)]
    L.tlim_hyperbolic_dt.argtypes = [vp, C.c_double, dp]
    L.tlim_status_str.argtypes = [C.c_int]
    L.tlim_last_error.restype = C.c_char_p
    L.tlim_last_error.argtypes = [vp]
    L.tlim_spectral_bound_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(Phase), C.c_int32, C.c_double, vp, vp, vp,
                                              vp, vp, vp, vp]
    for name in EXPORTED:
        if name != "tlim_status_str" and name != "tlim_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


@dataclass
class StepOpts:
    dt: float
    passes: int = 3
    picard_tol: float = 0.0
    order: int = ORDER_INTERLEAVED
    face_mean: int = FACE_ARITH
    cycle_mode: int = 0
    cycle_tol: float = 1e-13
    max_cycles: int = 200
    alpha_eps: float = 1e-10
    do_viscous: int = 0
    frozen_lambda: Optional[Sequence[float]] = None
    frozen_visc: Optional[Sequence[float]] = None
    time_sweeps: int = 0
    visc_heating: int = 0
    whole_step: int = 0
    _keep: list = dc_field(default_factory=list, repr=False)

    def c(self) -> StepOptsC:
        o = StepOptsC()
        for k in ("dt", "passes", "picard_tol", "order", "face_mean", "cycle_mode", "cycle_tol",
                  "max_cycles", "alpha_eps", "do_viscous", "time_sweeps", "visc_heating",
                  "whole_step"):
            setattr(o, k, getattr(self, k))
        self._keep = []
        for name in ("frozen_lambda", "frozen_visc"):
            vals = getattr(self, name)
            if vals is not None:
                arr = (C.c_double * len(vals))(*[float(x) for x in vals])
                self._keep.append(arr)
                setattr(o, name, C.cast(arr, C.POINTER(C.c_double)))
        return o


def _report(r: ReportC) -> dict:
    n = r.passes_run
    return dict(passes_run=n, converged=bool(r.converged), P=list(r.P[:n]),
                lambda_G=list(r.lambda_G[:n]), err=list(r.err[:n]), cycles=list(r.cycles[:n]),
                residual=list(r.residual[:n]), visc_P=list(r.visc_P),
                visc_lambda_G=list(r.visc_lambda_G), energy_before=r.energy_before,
                energy_after=r.energy_after, sweeps=r.sweeps, sweep_launches=r.sweep_launches,
                sweep_ms=r.sweep_ms, bad_cells=r.bad_cells, predicted=bool(r.predicted),
                mispredicted=bool(r.mispredicted), pipelined_steps=r.pipelined_steps,
                pipeline_redos=r.pipeline_redos, timed_sweeps=r.timed_sweeps, timed_launches=r.timed_launches)


class Solver:
    """One grid on one HIP device; fields live in a torch-allocated workspace."""

    def __init__(self, n, h=None, bc=None, precision: str = "fp64", device=None, stream=None):
        L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("tlim needs a HIP device (torch.cuda.is_available() is False)")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        g = make_grid(n, h, bc)
        n, h, bc = tuple(g.n), tuple(g.h), tuple(g.bc)
        self.n, self.h, self.bc = n, h, bc
        self.shape = (n[2], n[1], n[0])
        self.N = n[0] * n[1] * n[2]
        self.precision = FP32 if precision in ("fp32", FP32) else FP64
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            ctx = C.c_void_p()
            st = L.tlim_create(C.byref(g), self.precision, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
            if st != OK:
                raise TlimError(st, f"tlim_create failed: {L.tlim_status_str(st).decode()}")
            self._ctx = ctx
            nbytes = C.c_size_t()
            self._check(L.tlim_workspace_bytes(ctx, C.byref(nbytes)))
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self._check(L.tlim_bind_workspace(ctx, C.c_void_p(self.workspace.data_ptr()), nbytes.value))
        self._adj_ws = None
        _live.add(self)

    # -------------------------------------------------------------- basics
    def _check(self, st):
        if st != OK:
            L = load_library()
            msg = L.tlim_last_error(self._ctx).decode() if getattr(self, "_ctx", None) else ""
            raise TlimError(st, f"{L.tlim_status_str(st).decode()}: {msg}")

    def close(self):
        """Destroy the context (completing a pending step) and drop the
        workspace; the Solver is unusable afterwards."""
        if getattr(self, "_ctx", None):
            load_library().tlim_destroy(self._ctx)
            self._ctx = None
            self.workspace = None
            self._adj_ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_phase(self, k: int, p: dict):
        ph = make_phases([p, p])
        self._check(load_library().tlim_set_phase(self._ctx, int(k), C.byref(ph[0])))

    def _dev(self, t) -> torch.Tensor:
        t = torch.as_tensor(t)
        if t.dtype not in _DTYPES:
            t = t.to(torch.float64)
        t = t.to(self.device).contiguous()
        if t.numel() != self.N:
            raise ValueError(f"field has {t.numel()} values, grid has {self.N}")
        return t

    def set_field(self, name: str, values):
        """Copy a field in (float64 or float32 values; other types are
        converted to float64 first)."""
        t = self._dev(values)
        self._check(load_library().tlim_set_field(self._ctx, FIELDS[name], C.c_void_p(t.data_ptr()),
                                                  _DTYPES[t.dtype]))
        self.stream.synchronize()

    def clear_field(self, name: str) -> None:
        """Mark an optional field (u, v, w, src1, src2, E) as not set."""
        self._check(load_library().tlim_clear_field(self._ctx, FIELDS[name]))

    def get_field(self, name: str, dtype=torch.float64) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=dtype, device=self.device)
        self._check(load_library().tlim_get_field(self._ctx, FIELDS[name], C.c_void_p(out.data_ptr()),
                                                  _DTYPES[dtype]))
        self.stream.synchronize()
        return out

    def set_workload(self, wl: dict):
        """Phases and fields of a workload dict (paper_2106_00282_amd.workloads)."""
        for k in range(2):
            self.set_phase(k, wl["phases"][k])
        for name, arr in wl["fields"].items():
            self.set_field(name, torch.tensor(arr))

    # ------------------------------------------------------------ stepping
    def spectral_bound(self, face_mean: int = FACE_ARITH, alpha_eps: float = 1e-10) -> float:
        lam = C.c_double()
        self._check(load_library().tlim_spectral_bound(self._ctx, face_mean, alpha_eps, C.byref(lam)))
        return lam.value

    def advance(self, opts: StepOpts, report: bool = True):
        rep = ReportC()
        oc = opts.c()
        st = load_library().tlim_advance_parabolic(self._ctx, C.byref(oc), C.byref(rep) if report else None)
        if st not in (OK, E_NOCONV, E_NUMERIC):
            self._check(st)
        return st, (_report(rep) if report else None)

    def advance_hyperbolic(self, dt: float, relax_pressure: bool = True, report: bool = True):
        """One step of the hyperbolic part and the pressure relaxation
        (tlim_advance_hyperbolic).  Returns (status, bad_cells or None)."""
        o = HypOptsC(float(dt), int(bool(relax_pressure)))
        rep = HypReportC()
        st = load_library().tlim_advance_hyperbolic(self._ctx, C.byref(o), C.byref(rep) if report else None)
        if st not in (OK, E_NUMERIC):
            self._check(st)
        return st, (rep.bad_cells if report else None)

    def hyperbolic_dt(self, cfl: float) -> float:
        dt = C.c_double()
        self._check(load_library().tlim_hyperbolic_dt(self._ctx, float(cfl), C.byref(dt)))
        return dt.value

    def advance_raw(self, oc: StepOptsC) -> int:
        """Advance with a prepared options struct and no report (timing
        loops).  Predicted steps may stay pending (pipelined): finish()
        completes them."""
        return load_library().tlim_advance_parabolic(self._ctx, C.byref(oc), None)

    def finish(self) -> int:
        """Complete a pending pipelined step; returns its status."""
        return load_library().tlim_finish(self._ctx)

    # ------------------------------------------------------------- adjoint
    def forward_checkpointed(self, opts: StepOpts, nsteps: int, ckpt_every: int = 1):
        nck = (nsteps + ckpt_every - 1) // ckpt_every
        ckpt = torch.empty((nck,) + self.shape, dtype=torch.float64, device=self.device)
        lam = (C.c_double * (nsteps * opts.passes))()
        oc = opts.c()
        self._check(load_library().tlim_forward_checkpointed(self._ctx, C.byref(oc), nsteps, ckpt_every,
                                                             C.c_void_p(ckpt.data_ptr()), lam))
        return ckpt, [lam[i] for i in range(nsteps * opts.passes)]

    def adjoint_workspace(self, opts: StepOpts, nsteps: int, ckpt_every: int, lam, keep_interval=None) -> int:
        """Allocate (or keep) the adjoint's device workspace for this schedule;
        returns its size in bytes.  keep_interval: True sizes it for the layout
        that keeps every step of a checkpoint interval (no step recomputed
        twice), False for the one that keeps one step, None for the first when
        it fits in free device memory with a 10% margin.  A workspace already
        held is kept when large enough, and the adjoint takes the layout its
        size allows (both give the same result, bit for bit)."""
        L = load_library()
        lam_arr = (C.c_double * len(lam))(*[float(x) for x in lam])
        oc = opts.c()
        nbytes = C.c_size_t()
        self._check(L.tlim_adjoint_workspace_bytes(self._ctx, C.byref(oc), nsteps, lam_arr, C.byref(nbytes)))
        need = int(nbytes.value)
        if keep_interval is not False and min(ckpt_every, nsteps) > 1:
            kept = C.c_size_t()
            self._check(L.tlim_adjoint_workspace_bytes_kept(self._ctx, C.byref(oc), nsteps, ckpt_every, lam_arr,
                                                            C.byref(kept)))
            have = 0 if self._adj_ws is None else self._adj_ws.numel()
            if keep_interval:
                need = int(kept.value)
            elif have < kept.value:
                torch.cuda.empty_cache()
                free, _ = torch.cuda.mem_get_info(self.device)
                if kept.value - have <= 0.9 * free:
                    need = int(kept.value)
            else:
                need = int(kept.value)
        if self._adj_ws is None or self._adj_ws.numel() < need:
            self._adj_ws = None
            self._adj_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._adj_ws.numel()

    def adjoint(self, opts: StepOpts, nsteps: int, ckpt_every: int, ckpt: torch.Tensor, lam, dL_dTN,
                keep_interval=None):
        """dL/dT^0 and dL/dk0 from dL/dT^N (see adjoint_workspace for
        keep_interval; a workspace already large enough is reused)."""
        L = load_library()
        lam_arr = (C.c_double * len(lam))(*[float(x) for x in lam])
        oc = opts.c()
        self.adjoint_workspace(opts, nsteps, ckpt_every, lam, keep_interval)
        g = self._dev(dL_dTN)
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        dk0 = (C.c_double * 2)()
        self._check(L.tlim_adjoint_parabolic(self._ctx, C.byref(oc), nsteps, ckpt_every, C.c_void_p(ckpt.data_ptr()),
                                   lam_arr, C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()), dk0,
                                   C.c_void_p(self._adj_ws.data_ptr()), self._adj_ws.numel()))
        return out, [dk0[0], dk0[1]]


def make_grid(n, h=None, bc=None) -> Grid:
    """tlim_grid of n = (nx[, ny[, nz]]) cells; h defaults to the unit box's
    spacing, bc to periodic axes."""
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


def make_phases(phases) -> "C.Array":
    """tlim_phase[2] from two dicts (keys of tlim_phase; missing ones 0, T0 1)."""
    arr = (Phase * 2)()
    for k in range(2):
        p = phases[k]
        for name in ("gamma", "pinf", "cv", "q", "k0", "T0", "npow", "mu"):
            setattr(arr[k], name, float(p.get(name, 1.0 if name == "T0" else 0.0)))
        arr[k].law = int(p.get("law", LAW_POWER))
        for name in ("sh_D", "sh_LD", "sh_dB"):
            setattr(arr[k], name, float(p.get(name, 0.0)))
    return arr


def spectral_bound_noalloc(grid: Grid, phases, alpha2, m1, m2, T1, T2, out, face_mean: int = FACE_ARITH,
                           alpha_eps: float = 1e-10, stream=None) -> None:
    """tlim_spectral_bound_noalloc: the bound of the relaxed fields (float64
    device tensors, contiguous) into out[0] (a float64 device tensor), queued
    on `stream` (default: the current stream); no allocation, no
    synchronisation."""
    L = load_library()
    for t in (alpha2, m1, m2, T1, T2, out):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("fields and out must be contiguous float64 device tensors")
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    ph = make_phases(phases)
    r = L.tlim_spectral_bound_noalloc(C.byref(grid), ph, int(face_mean), float(alpha_eps),
                                      *[C.c_void_p(t.data_ptr()) for t in (alpha2, m1, m2, T1, T2, out)],
                                      C.c_void_p(st.cuda_stream))
    if r != OK:
        raise TlimError(r, f"{L.tlim_status_str(r).decode()}: {L.tlim_last_error(None).decode()}")


class ParabolicRun(torch.autograd.Function):
    """T^N = (nsteps heat steps)(T^0; k0) with a hand-written adjoint.

    forward(T0, k0, solver, opts, nsteps, ckpt_every, phases): sets k0 of both
    phases and T1 = T2 = T0 on ``solver`` (whose alpha2, m1, m2 are already
    set), runs the checkpointed forward and returns T^N.  backward recomputes
    each step from its checkpoint and reverses it (tlim_adjoint_parabolic)."""

    @staticmethod
    def forward(ctx, T0, k0, solver: Solver, opts: StepOpts, nsteps: int, ckpt_every: int, phases):
        phases = [dict(p) for p in phases]
        for k in range(2):
            phases[k]["k0"] = float(k0[k])
            solver.set_phase(k, phases[k])
        solver.set_field("T1", T0.detach())
        solver.set_field("T2", T0.detach())
        ckpt, lam = solver.forward_checkpointed(opts, nsteps, ckpt_every)
        ctx.solver, ctx.opts, ctx.nsteps, ctx.ckpt_every = solver, opts, nsteps, ckpt_every
        ctx.ckpt, ctx.lam = ckpt, lam
        ctx.k0_dtype, ctx.k0_device = k0.dtype, k0.device
        return solver.get_field("T1").reshape(T0.shape)

    @staticmethod
    def backward(ctx, grad_out):
        dT0, dk0 = ctx.solver.adjoint(ctx.opts, ctx.nsteps, ctx.ckpt_every, ctx.ckpt, ctx.lam,
                                      grad_out.detach().to(torch.float64))
        gk0 = torch.tensor(dk0, dtype=ctx.k0_dtype, device=ctx.k0_device)
        return dT0.reshape(grad_out.shape).to(grad_out.dtype), gk0, None, None, None, None, None
