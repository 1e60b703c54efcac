"""Seeded synthetic two-phase workloads.

This module only builds inputs: grids, material constants and initial
fields.  It holds none of the method's arithmetic (no coefficients, no
spectral bound, no time step) and serves the GPU path, the oracle and the
benchmark alike.  The time step of a workload is given as a multiple ``dt_factor``
of the explicit stability limit 2/lambda_G of the initial post-relaxation
state; whoever runs the workload evaluates lambda_G with its own code.

Arrays are float64, C-contiguous, shaped (nz, ny, nx) with x fastest, on the
unit box with cell centres at (i + 1/2) h.

Materials (every workload): ideal gases (p_inf = q = 0), rho = (1, 10),
C_v = (1, 0.5) so rho*C_v = (1, 5), gamma = (3.0, 1.4) so that
(gamma_k - 1) rho_k C_v,k is the same for both phases and an initial state
with T_1 = T_2 is in pressure equilibrium.  Conductivity
lambda_k(T) = k0_k (T/T0)^n with T0 = 1.

Workloads (sizes are parameters; the defaults are the full sizes):
  heat1d     1024 cells, adiabatic; alpha_1 = (1 - tanh((x-1/2)/(3h)))/2,
             k = (1, 0.1) constant, T = 2 left of 1/2 and 1 right; one
             step at 100x the explicit limit.
  levelset2d 1024^2 periodic; alpha_1 = (1 - tanh(phi/(2h)))/2 of a level set
             of 8 random sinusoids with wavenumbers 1..6 scaled to unit
             gradient; T lognormal (sigma 0.2) about 1; k0 = (1, 0.05),
             n = 2; 10 steps at 200x, 3 Picard passes.
  bubbles3d  256^3 periodic, 20 spheres of radius 10..30 cells (of a 256
             grid) of phase 2 with a temperature jump of up to 2x and a
             smooth velocity bump each; viscosity (1e-2, 1e-3); 5 steps.
  levelset2d_adjoint  the level-set generator at 2048^2, 20 steps, loss
             against a target made with k0 scaled by 1.1.
  interface3d  512^3, x adiabatic, y and z periodic; planar interface at
             x = 1/2 perturbed by 12 cosine modes of amplitude 5 cells;
             k0 = (1, 0.01); T = 1 + alpha_1; 10 steps.
  interface1d  the interface translation of Sec. 4.1 (PVT property): 1 m,
             SG liquid (gamma 4.4, C_v 500, p_inf 6e8) left of x = 0.2 and
             ideal gas (gamma 1.4, C_v 200) right of it, tanh profile of
             width 2 cells, alpha clipped to [1e-6, 1 - 1e-6], u = 1000,
             p = 1e5, T = 300 in both phases; periodic.
  shocktube2d  hyperbolic workload, 1024^2 periodic: the level-set
             interface of levelset2d between a gas (gamma 1.4, rho 1) and a
             stiffened liquid (gamma 4.4, p_inf 10, rho 10), alpha clipped to
             [1e-6, 1 - 1e-6], at rest, with pressure 10 in the band
             0.25 < x < 0.5 and 1 elsewhere (T_k from p and rho_k); steps at
             CFL 0.4.
  levelset2d_spitzer  the level-set fields with the Spitzer-Harm law for
             both phases: n = 5/2, Coulomb-log lengths l_D = e^2.5 sqrt(T/rho),
             l_LD = 1/T, l_dB = 1/sqrt(T), so that the Landau branch holds
             below T = 1, the de Broglie branch above it, and the floor
             ln Lambda = 1 in the cold dense cells; 10 steps at 200x.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 210600282
PERIODIC, ADIABATIC = 0, 1
LAW_POWER, LAW_SPITZER = 0, 1


def base_phases(k0=(1.0, 0.05), npow=2.0, mu=(0.0, 0.0)):
    rho = (1.0, 10.0)
    cv = (1.0, 0.5)
    gamma = (3.0, 1.4)
    return [dict(gamma=gamma[k], pinf=0.0, cv=cv[k], q=0.0, k0=k0[k], T0=1.0, npow=npow,
                 mu=mu[k], rho=rho[k]) for k in range(2)]


def spitzer_phases(phases, sh_D=float(np.exp(2.5)), sh_LD=1.0, sh_dB=1.0, npow=2.5):
    """Copies of ``phases`` switched to the Spitzer-Harm law with the given
    Coulomb-log length constants (l_D = sh_D sqrt(T/rho), l_LD = sh_LD/T,
    l_dB = sh_dB/sqrt(T))."""
    out = []
    for p in phases:
        q = dict(p)
        q.update(law=LAW_SPITZER, npow=float(npow), sh_D=float(sh_D), sh_LD=float(sh_LD),
                 sh_dB=float(sh_dB))
        out.append(q)
    return out


def _streams(config_id: int, n: int):
    ss = np.random.SeedSequence(SEED_BASE + config_id)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def _centres(n: int):
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _finish(name, n, bc, phases, alpha1, T, dt_factor, steps, passes, vel=None, extra=None):
    alpha1 = np.ascontiguousarray(alpha1, dtype=np.float64)
    alpha2 = np.ascontiguousarray(1.0 - alpha1)
    rho = [p["rho"] for p in phases]
    fields = dict(alpha2=alpha2,
                  m1=np.ascontiguousarray(alpha1 * rho[0]),
                  m2=np.ascontiguousarray(alpha2 * rho[1]),
                  T1=np.ascontiguousarray(T, dtype=np.float64),
                  T2=np.ascontiguousarray(T, dtype=np.float64).copy())
    if vel is not None:
        for key, arr in zip(("u", "v", "w"), vel):
            if arr is not None:
                fields[key] = np.ascontiguousarray(arr, dtype=np.float64)
    h = tuple(1.0 / x if x > 1 else 1.0 for x in n)
    wl = dict(name=name, n=tuple(n), h=h, bc=tuple(bc), phases=phases, fields=fields,
              dt_factor=float(dt_factor), steps=int(steps), passes=int(passes),
              viscous=vel is not None)
    if extra:
        wl.update(extra)
    return wl


def heat1d(nx: int = 1024):
    """Two-phase 1D conduction: one implicit step at 100x the explicit limit."""
    phases = base_phases(k0=(1.0, 0.1), npow=0.0)
    x = _centres(nx)
    h = 1.0 / nx
    alpha1 = 0.5 * (1.0 - np.tanh((x - 0.5) / (3.0 * h)))
    T = np.where(x < 0.5, 2.0, 1.0)
    return _finish("heat1d", (nx, 1, 1), (ADIABATIC, PERIODIC, PERIODIC), phases,
                   alpha1.reshape(1, 1, nx), T.reshape(1, 1, nx), 100.0, 1, 1)


def _levelset_fields(n: int, config_id: int):
    rs_modes, rs_T = _streams(config_id, 2)
    amp = rs_modes.uniform(0.5, 1.0, size=8)
    kx = rs_modes.integers(1, 7, size=8) * rs_modes.choice([-1, 1], size=8)
    ky = rs_modes.integers(1, 7, size=8) * rs_modes.choice([-1, 1], size=8)
    theta = rs_modes.uniform(0.0, 2.0 * np.pi, size=8)
    x = _centres(n)[None, :]
    y = _centres(n)[:, None]
    phi = np.zeros((n, n))
    gx = np.zeros((n, n))
    gy = np.zeros((n, n))
    for j in range(8):
        arg = 2.0 * np.pi * (kx[j] * x + ky[j] * y) + theta[j]
        phi += amp[j] * np.sin(arg)
        c = amp[j] * np.cos(arg) * 2.0 * np.pi
        gx += c * kx[j]
        gy += c * ky[j]
    phi /= np.sqrt(gx * gx + gy * gy).max()
    h = 1.0 / n
    alpha1 = 0.5 * (1.0 - np.tanh(phi / (2.0 * h)))
    T = np.exp(0.2 * rs_T.standard_normal((n, n)))
    return alpha1.reshape(1, n, n), T.reshape(1, n, n)


def levelset2d(n: int = 1024, steps: int = 10):
    """2D periodic two-phase conduction with T^2 conductivities, 200x limit."""
    phases = base_phases(k0=(1.0, 0.05), npow=2.0)
    alpha1, T = _levelset_fields(n, 2)
    return _finish("levelset2d", (n, n, 1), (PERIODIC,) * 3, phases, alpha1, T, 200.0, steps, 3)


def levelset2d_spitzer(n: int = 1024, steps: int = 10):
    """The level-set workload with Spitzer-Harm conductivities (both phases)."""
    phases = spitzer_phases(base_phases(k0=(1.0, 0.05)))
    alpha1, T = _levelset_fields(n, 2)
    return _finish("levelset2d_spitzer", (n, n, 1), (PERIODIC,) * 3, phases, alpha1, T, 200.0,
                   steps, 3)


def _sg_state(phases, alpha2, rho, p, vel):
    """Library fields from alpha_2, phase densities, a common pressure and a
    velocity: T_k = (p + p_inf,k) / ((gamma_k - 1) rho_k C_v,k), the SG EOS
    read at the given density and pressure (input construction only)."""
    a2 = np.ascontiguousarray(alpha2, dtype=np.float64)
    f = dict(alpha2=a2, m1=np.ascontiguousarray((1.0 - a2) * rho[0]), m2=np.ascontiguousarray(a2 * rho[1]))
    for k in range(2):
        ph = phases[k]
        T = (p + ph["pinf"]) / ((ph["gamma"] - 1.0) * rho[k] * ph["cv"])
        f[f"T{k + 1}"] = np.ascontiguousarray(np.broadcast_to(T, a2.shape), dtype=np.float64)
    for key, v in zip(("u", "v", "w"), vel):
        f[key] = np.ascontiguousarray(np.broadcast_to(v, a2.shape), dtype=np.float64)
    return f


def interface1d(n: int = 1000, steps: int = 100):
    """Interface translation in uniform p, u, T (Sec. 4.1)."""
    phases = [dict(gamma=4.4, pinf=6e8, cv=500.0, q=0.0, k0=0.0, T0=1.0, npow=0.0, mu=0.0),
              dict(gamma=1.4, pinf=0.0, cv=200.0, q=0.0, k0=0.0, T0=1.0, npow=0.0, mu=0.0)]
    x = _centres(n)
    a2 = (0.5 * (1.0 + np.tanh((x - 0.2) / (2.0 / n)))).clip(1e-6, 1.0 - 1e-6).reshape(1, 1, n)
    p, T = 1e5, 300.0
    rho = [(p + 6e8) / (3.4 * 500.0 * T), p / (0.4 * 200.0 * T)]
    f = _sg_state(phases, a2, rho, p, (1000.0, 0.0, 0.0))
    return dict(name="interface1d", n=(n, 1, 1), h=(1.0 / n, 1.0, 1.0), bc=(PERIODIC,) * 3, phases=phases,
                fields=f, steps=int(steps), cfl=0.5, T=T, p=p, u=1000.0)


def shocktube2d(n: int = 1024, steps: int = 10):
    """Hyperbolic workload: a pressure band crossing a level-set interface."""
    phases = [dict(gamma=1.4, pinf=0.0, cv=1.0, q=0.0, k0=1.0, T0=1.0, npow=0.0, mu=0.0),
              dict(gamma=4.4, pinf=10.0, cv=0.5, q=0.0, k0=0.05, T0=1.0, npow=0.0, mu=0.0)]
    alpha1, _ = _levelset_fields(n, 6)
    a2 = (1.0 - alpha1).clip(1e-6, 1.0 - 1e-6)
    x = _centres(n)[None, None, :]
    p = np.where((x > 0.25) & (x < 0.5), 10.0, 1.0) * np.ones_like(a2)
    f = _sg_state(phases, a2, (1.0, 10.0), p, (0.0, 0.0, 0.0))
    return dict(name="shocktube2d", n=(n, n, 1), h=(1.0 / n, 1.0 / n, 1.0), bc=(PERIODIC,) * 3, phases=phases,
                fields=f, steps=int(steps), cfl=0.4)


def levelset2d_adjoint(n: int = 2048, steps: int = 20):
    """The level-set workload with a misfit loss for the adjoint: target made
    with k0 scaled by 1.1 (both phases), same initial fields and time step."""
    phases = base_phases(k0=(1.0, 0.05), npow=2.0)
    alpha1, T = _levelset_fields(n, 2)
    rs = _streams(4, 1)[0]
    N = n * n
    probe = rs.choice(N, size=16, replace=False)
    return _finish("levelset2d_adjoint", (n, n, 1), (PERIODIC,) * 3, phases, alpha1, T, 200.0,
                   steps, 3, extra=dict(target_k0_scale=1.1, fd_cells=np.sort(probe)))


def bubbles3d(n: int = 256, steps: int = 5, nbubbles: int = 20, shape=None):
    """3D periodic bubbles with temperature jumps and velocity, plus viscosity.
    shape = (nx, ny, nz) gives a box of other proportions on the same unit
    cube (spacing 1/n per axis; the interface width is 2 cells of x)."""
    phases = base_phases(k0=(1.0, 0.05), npow=2.0, mu=(1e-2, 1e-3))
    rs_c, rs_r, rs_J, rs_u = _streams(3, 4)
    centres = rs_c.uniform(0.0, 1.0, size=(nbubbles, 3))
    radii = rs_r.uniform(10.0, 30.0, size=nbubbles) / 256.0
    jumps = rs_J.uniform(1.0, 2.0, size=nbubbles)
    uvec = 0.1 * rs_u.uniform(-1.0, 1.0, size=(nbubbles, 3))
    nx, ny, nz = shape if shape is not None else (n, n, n)
    h = 1.0 / nx
    cx, cy, cz = _centres(nx), _centres(ny), _centres(nz)
    alpha2 = np.zeros((nz, ny, nx))
    Tbump = np.zeros((nz, ny, nx))
    vel = [np.zeros((nz, ny, nx)) for _ in range(3)]
    for b in range(nbubbles):
        # periodic distance along each axis (z, y, x order of the array)
        dz = np.abs(cz - centres[b, 2]); dz = np.minimum(dz, 1.0 - dz)
        dy = np.abs(cy - centres[b, 1]); dy = np.minimum(dy, 1.0 - dy)
        dx = np.abs(cx - centres[b, 0]); dx = np.minimum(dx, 1.0 - dx)
        r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        s = 0.5 * (1.0 - np.tanh((r - radii[b]) / (2.0 * h)))
        np.maximum(alpha2, s, out=alpha2)
        np.maximum(Tbump, (jumps[b] - 1.0) * s, out=Tbump)
        for d in range(3):
            vel[d] += uvec[b, d] * s
    T = 1.0 + Tbump
    return _finish("bubbles3d", (nx, ny, nz), (PERIODIC,) * 3, phases, 1.0 - alpha2, T, 200.0,
                   steps, 3, vel=vel)


def interface3d(n: int = 512, steps: int = 10, nmodes: int = 12, shape=None):
    """3D perturbed planar interface, conductivity contrast 100.  shape =
    (nx, ny, nz) gives a box of other proportions (spacing 1/n per axis, the
    modes stay periodic in y and z, amplitude 5 cells of x)."""
    phases = base_phases(k0=(1.0, 0.01), npow=2.0)
    rs = _streams(5, 1)[0]
    modes = []
    while len(modes) < nmodes:
        m, q = (int(v) for v in rs.integers(0, 7, size=2))
        if (m, q) != (0, 0) and (m, q) not in modes:
            modes.append((m, q))
    amp = rs.uniform(0.5, 1.0, size=nmodes)
    theta = rs.uniform(0.0, 2.0 * np.pi, size=nmodes)
    nx, ny, nz = shape if shape is not None else (n, n, n)
    h = 1.0 / nx
    y = _centres(ny)[:, None]
    z = _centres(nz)[None, :]
    pert = np.zeros((ny, nz))
    for j, (m, q) in enumerate(modes):
        pert += amp[j] * np.cos(2.0 * np.pi * (m * y + q * z) + theta[j])
    pert *= 5.0 * h / np.abs(pert).max()
    xint = 0.5 + pert  # indexed (y, z)
    x = _centres(nx)
    alpha1 = np.empty((nz, ny, nx))
    for k in range(nz):
        alpha1[k] = 0.5 * (1.0 - np.tanh((x[None, :] - xint[:, k][:, None]) / (2.0 * h)))
    T = 1.0 + alpha1
    return _finish("interface3d", (nx, ny, nz), (ADIABATIC, PERIODIC, PERIODIC), phases, alpha1, T,
                   200.0, steps, 3)


WORKLOADS = dict(heat1d=heat1d, levelset2d=levelset2d, bubbles3d=bubbles3d,
                 levelset2d_adjoint=levelset2d_adjoint, interface3d=interface3d)


def random_case(seed: int):
    """A small random two-phase workload for property-style parity runs:
    1D, 2D or 3D, random sizes and boundary conditions, random phase
    constants (equal p_inf = 0, conductivity exponents including non-integer
    ones, about a third with the Spitzer-Harm Coulomb logarithm), a smooth random interface with some pure cells, phase
    temperatures out of equilibrium, dt between 1x and 300x the explicit
    limit and 1-3 Picard passes."""
    rs = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 7, seed])))
    dim = int(rs.integers(1, 4))
    if dim == 1:
        n = (int(rs.integers(3, 300)), 1, 1)
    elif dim == 2:
        n = (int(rs.integers(2, 160)), int(rs.integers(2, 160)), 1)
    else:
        n = (int(rs.integers(2, 24)), int(rs.integers(2, 24)), int(rs.integers(2, 24)))
    bc = tuple(int(rs.integers(0, 2)) if n[d] > 1 else PERIODIC for d in range(3))
    npow = float(rs.choice([0.0, 1.0, 2.0, 2.5, 3.0, 1.7]))
    phases = []
    for k in range(2):
        phases.append(dict(gamma=float(rs.uniform(1.2, 3.0)), pinf=0.0, cv=float(rs.uniform(0.3, 2.0)), q=0.0,
                           k0=float(10 ** rs.uniform(-2, 0.5)), T0=float(rs.uniform(0.5, 2.0)), npow=npow,
                           mu=0.0, rho=float(10 ** rs.uniform(-0.5, 1.0))))
    shape = (n[2], n[1], n[0])
    coords = np.meshgrid(*[_centres(n[d]) for d in (2, 1, 0)], indexing="ij")  # z, y, x
    phi = np.zeros(shape)
    for _ in range(4):
        kvec = rs.integers(0, 4, size=3)
        amp = rs.uniform(0.2, 1.0)
        phase = rs.uniform(0, 2 * np.pi)
        phi += amp * np.cos(2 * np.pi * (kvec[0] * coords[2] + kvec[1] * coords[1] + kvec[2] * coords[0]) + phase)
    alpha1 = 0.5 * (1.0 - np.tanh(phi * rs.uniform(2.0, 8.0)))
    alpha1[alpha1 < 0.02] = 0.0
    alpha1[alpha1 > 0.98] = 1.0
    T = np.exp(0.3 * rs.standard_normal(shape))
    wl = _finish(f"random{seed}", n, bc, phases, alpha1, T, float(rs.uniform(1.0, 300.0)), 2,
                 int(rs.integers(1, 4)))
    wl["fields"]["T2"] = np.ascontiguousarray(wl["fields"]["T1"] * np.exp(0.1 * rs.standard_normal(shape)))
    # drawn last, so that the fields above do not depend on it
    if rs.uniform() < 0.35:
        wl["phases"] = spitzer_phases(phases, sh_D=float(np.exp(rs.uniform(1.0, 3.5))),
                                      sh_LD=float(np.exp(rs.uniform(-0.5, 0.5))),
                                      sh_dB=float(np.exp(rs.uniform(-0.5, 0.5))), npow=npow)
    return wl
