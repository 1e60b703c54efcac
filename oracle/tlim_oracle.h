/*
 * FP64 CPU oracle for the parabolic sub-step (heat conduction + viscosity)
 * of the two-temperature diffuse-interface model of Zhang, Menshov, Wang and
 * Shen, "Diffuse interface relaxation model for two-phase compressible flows
 * with diffusion processes" (arXiv 2106.00282).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code; only the tests, the smoke check and the CPU baseline of
 * the benchmark do.  It shares no source with the GPU library.
 *
 * Plain scalar loops, double precision throughout, steps taken in the order
 * the paper gives them:
 *   - temperature relaxation in mixed cells      (Sec. 3.4.1, eqs. ht_eq2_TR_dis,
 *                                                 ht_eq3_TR_dis, Taverage)
 *   - heat-conduction coefficients and the
 *     central-difference operator                (Sec. 3.4.2, eq. qk_dis)
 *   - method of local iterations (LIM)           (Sec. 3.2, eqs. LIM, LIM_last)
 *   - Picard loop with volume-fraction update    (Algorithm 1)
 *   - viscous momentum diffusion                 (Sec. 3.2, eq. viscous1D)
 *   - Chebyshev cycles to the backward-Euler
 *     solution ("cycle mode") and its adjoint
 *   - the power and Spitzer-Harm conductivity
 *     laws                                       (Sec. 3.4.2, Sec. 4.4)
 *   - the hyperbolic part, Godunov method with
 *     HLLC faces, and the pressure relaxation    (Sec. 3.1, eq. vectorForm;
 *                                                 Sec. 3.3)
 *
 * Pinned by the CPU tests: closed-form Fourier multiplier of one LIM pass,
 * brute-force backward Euler, Chebyshev cycle rate, energy conservation,
 * maximum principle, PVT invariance, relaxation closed forms, Picard
 * invariance for constant conductivity, adjoint vs finite differences and
 * the dot-product identity; the Spitzer-Harm law's worked values,
 * log-derivatives and floor; for the hyperbolic part the Euler HLLC
 * reduction, conservation, interface translation, volume-fraction
 * advection, wall symmetry and the ideal-gas closed form of the pressure
 * relaxation.  The heat step of two stiffened gases with unequal p_inf
 * (effective capacity and volume-fraction update) is pinned from the
 * equation of state alone: under a uniform source it reaches the exact
 * end state (energy E0 + tau I, p_1 = p_2) with an O(tau^2) error; with
 * conduction on one explicit stage every cell's EOS energy changes by tau
 * times the net flux of eq. qk_dis and the pressure gap is O(tau^2); at
 * tau lambda = 400 the domain's EOS energy is conserved.
 *
 * The nonlinear-conductivity Picard result has no closed form; it is
 * pinned as the fixed point of the lagged pass: at convergence T* equals one
 * LIM pass from T^n at Lambda(T*), evaluated through the eigendecomposition
 * of the symmetric operator and the pass's closed-form multiplier.
 *
 * Parity unpinned: the split of the internal energy between two different
 * phases across a wave of the hyperbolic part is held only through the
 * mixture, the advection of alpha_2, the interface translation and the
 * interchangeability of the phase labels.
 */
#ifndef TLIM_ORACLE_H
#define TLIM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary condition per axis. */
enum { ORC_PERIODIC = 0, ORC_ADIABATIC = 1 };
/* Order of the Chebyshev parameters inside one LIM pass. */
enum { ORC_ORDER_INTERLEAVED = 0, ORC_ORDER_PAPER = 1, ORC_ORDER_ASCENDING = 2 };
/* Face mean of the cell conductivities. */
enum { ORC_FACE_ARITH = 0, ORC_FACE_HARMONIC = 1 };

/* Cell-centred grid: n[0] cells along x (fastest), n[1] along y, n[2] along z.
 * Field index i + n0*(j + n1*k). */
typedef struct {
    int64_t n[3];
    double h[3];
    int32_t bc[3];
} orc_grid;

/* One phase: stiffened-gas EOS (gamma, p_inf, C_v, q), conductivity law,
 * dynamic viscosity mu.
 * law ORC_LAW_POWER:   lambda(T) = k0 * (T/T0)^npow.
 * law ORC_LAW_SPITZER: lambda(rho, T) = k0 * (T/T0)^npow / ln Lambda_ei(rho, T),
 *   the Spitzer-Harm form of Sec. 4.4 (npow = 5/2 there) with its Coulomb
 *   logarithm, from the Debye, Landau and de Broglie lengths
 *   l_D = sh_D sqrt(T/rho), l_LD = sh_LD / T, l_dB = sh_dB / sqrt(T);
 *   rho is the cell's mixture density m1 + m2. */
enum { ORC_LAW_POWER = 0, ORC_LAW_SPITZER = 1 };
typedef struct {
    double gamma, pinf, cv, q;
    double k0, T0, npow;
    double mu;
    int32_t law;
    double sh_D, sh_LD, sh_dB;
} orc_phase;

/* Options of one parabolic step. */
typedef struct {
    double tau;          /* time step */
    int32_t passes;      /* maximum number of Picard passes */
    double picard_tol;   /* stop when err < tol; 0 = always run all passes */
    int32_t order;       /* ORC_ORDER_* */
    int32_t face_mean;   /* ORC_FACE_* */
    int32_t cycle_mode;  /* 0 = one LIM pass per Picard pass; 1 = Chebyshev cycles to BE */
    double cycle_tol;    /* relative residual target of cycle mode */
    int32_t max_cycles;
    double alpha_eps;    /* mixed cell: eps < alpha2 < 1 - eps */
    int32_t do_viscous;  /* run the viscous sub-step first */
    int32_t visc_heating; /* viscous part also heats the phases (orc_visc_heat) */
} orc_opts;

/* Per-step report (filled by the step driver). */
#define ORC_MAX_PASSES 64
typedef struct {
    int32_t passes_run;
    int32_t converged;
    int32_t P[ORC_MAX_PASSES];
    double lambda_G[ORC_MAX_PASSES];
    double err[ORC_MAX_PASSES];
    int32_t cycles[ORC_MAX_PASSES];
    double residual[ORC_MAX_PASSES];
    int32_t visc_P[3];
    double visc_lambda_G[3];
    double energy_before, energy_after;
} orc_report;

/* ---- building blocks (exported for the pin tests) ---- */

/* Number of Chebyshev parameters P = ceil(pi/4 * sqrt(tau*lambda + 1)). */
int32_t orc_lim_P(double tau, double lambda_max);
/* Stage parameters b_1..b_{2P-1} of one LIM pass (last one is 0). */
void orc_lim_params(int32_t P, double lambda_max, int32_t order, double* b);
/* Stage parameters of one Chebyshev-Richardson cycle of s stages. */
void orc_cycle_params(int32_t s, double lambda_max, double* b);

/* Cell conductivity Lambda_i = sum_k alpha_k lambda_k(rho_i, T_i), rho_i = m1 + m2
 * (m1, m2 may be NULL when no phase uses the Spitzer-Harm law). */
void orc_cell_conductivity(const orc_grid* g, const orc_phase ph[2], const double* alpha2,
                           const double* m1, const double* m2, const double* T, double* Lam);
/* Effective heat capacity of the equilibrium heat step (per unit volume). */
void orc_heat_capacity(const orc_grid* g, const orc_phase ph[2], double eps,
                       const double* alpha2, const double* m1, const double* m2,
                       const double* T, double* C);
/* Gershgorin bound lambda_G = max_i 2 d_i of A = C^-1 D. */
double orc_gershgorin(const orc_grid* g, const double* Lam, const double* C,
                      const double axis_scale[3], int32_t face_mean);
/* y = A v = C^-1 D v. */
void orc_apply_A(const orc_grid* g, const double* Lam, const double* C,
                 const double axis_scale[3], int32_t face_mean,
                 const double* v, double* y);
/* One LIM pass: out = v^(nst) from v^(0) = v0 with right-hand side g.
 * The last stage (b = 0) is evaluated in conservative flux form.
 * If stages != NULL, v^(0..nst-1) are stored there (nst*N doubles). */
void orc_lim_pass(const orc_grid* g, const double* Lam, const double* C,
                  const double axis_scale[3], int32_t face_mean, double tau,
                  int32_t nst, const double* b, const double* rhs, const double* v0,
                  double* out, double* stages);

/* Viscous heating of the phases by one velocity component (Sec. 3.2, the
 * phase internal-energy update after the momentum pass).  uh is the
 * predicted velocity (after the first 2P-2 stages), mu the cell viscosity,
 * axis_scale the factors s_d of mu_cd (4/3 on the component's own axis).
 * T1, T2 are updated in place. */
void orc_visc_heat(const orc_grid* g, const orc_phase ph[2], double eps, int32_t face_mean,
                   const double* alpha2, const double* m1, const double* m2, const double* mu,
                   const double axis_scale[3], double tau, const double* uh, double* T1, double* T2);

/* Total-energy update of the viscous part by one velocity component (Sec.
 * 3.2): (rho E)_a changes by tau/h_d [uh_f+ F_f+ - uh_f- F_f-] summed over
 * the axes, with F and the face values as in orc_visc_heat.  E in place. */
void orc_visc_energy(const orc_grid* g, int32_t face_mean, const double* mu, const double axis_scale[3],
                     double tau, const double* uh, double* E);

/* Temperature relaxation in mixed cells (in place on alpha2, T1, T2). */
void orc_relax(const orc_grid* g, const orc_phase ph[2], double eps,
               double* alpha2, const double* m1, const double* m2,
               double* T1, double* T2);

/* Total internal energy sum_i vol*(sum_k C_k T_k + alpha_k p_inf_k). */
double orc_energy(const orc_grid* g, const orc_phase ph[2], const double* alpha2,
                  const double* m1, const double* m2, const double* T1, const double* T2);

/* ---- drivers ---- */

/* One parabolic step: [viscous], relaxation, Picard loop of LIM passes.
 * u, v, w may be NULL when do_viscous = 0.  src1/src2 may be NULL.
 * E (nullable) is the mixture total energy density rho E: the viscous part
 * adds orc_visc_energy per component, the heat part C_eff (T^{n+1} - T^n)
 * with the last pass's C_eff and the relaxed T^n -- the conductive flux
 * divergence plus the sources of that pass's final stage.
 * frozen_lambda (nullable, `passes` entries) replaces the Gershgorin bound of
 * each pass; frozen_visc (nullable, 3 entries) that of each velocity component.
 * Returns 0, or 3 when picard_tol > 0 was not reached. */
int32_t orc_step(const orc_grid* g, const orc_phase ph[2], const orc_opts* o,
                 double* alpha2, const double* m1, const double* m2,
                 double* T1, double* T2, const double* src1, const double* src2,
                 double* u, double* v, double* w, double* E,
                 const double* frozen_lambda, const double* frozen_visc,
                 orc_report* rep);

/* Chebyshev-Richardson cycles of s stages towards (I + tau A) v = rhs, from
 * v0, until the relative residual is below tol or max_cycles were run.
 * residual_hist (nullable) receives the residual after each cycle.
 * Returns the number of cycles run. */
int32_t orc_cycle_solve(const orc_grid* g, const double* Lam, const double* C,
                        const double axis_scale[3], int32_t face_mean, double tau,
                        double lambda_max, int32_t s, const double* rhs, const double* v0,
                        double tol, int32_t max_cycles, double* out, double* residual_hist);

/* Backward-Euler residual || C(g - v) - tau D v ||_2 / || C g ||_2. */
double orc_be_residual(const orc_grid* g, const double* Lam, const double* C,
                       const double axis_scale[3], int32_t face_mean, double tau,
                       const double* rhs, const double* v);

/* Adjoint of `nsteps` heat steps (equilibrium input, p_inf,1 = p_inf,2,
 * no viscous, no sources) with the frozen schedule lam[step*passes + pass].
 * Inputs: alpha2, m1, m2, initial T0, dL/dT^N.  Outputs dL/dT0 (N) and
 * dL/dk0 (2).  Also returns T^N in TN (nullable). */
int32_t orc_heat_adjoint(const orc_grid* g, const orc_phase ph[2], const orc_opts* o,
                         int32_t nsteps, const double* lam,
                         const double* alpha2, const double* m1, const double* m2,
                         const double* T0, const double* dL_dTN,
                         double* dL_dT0, double* dL_dk0, double* TN);

/* ---- hyperbolic part and pressure relaxation (Sec. 3.1, Sec. 3.3) ---- */

/* One first-order Godunov step of the hyperbolic part (eq. vectorForm, HLLC
 * faces, dimensional splitting x, y, z), each directional sweep followed,
 * if relax_pressure, by the pressure relaxation of every cell.  The state is updated in place: alpha2,
 * m_k, T_k (eq. eos_stiffened2), the velocity (u, v, w nullable = 0 and not
 * written) and rho E (E nullable: then taken from the state and not
 * written).  Adiabatic axes are reflecting walls.  Every cell must hold
 * both phases (0 < alpha2 < 1, m_k > 0).  Returns 1 if a cell left that
 * range or a temperature is not positive, else 0. */
int32_t orc_hyperbolic(const orc_grid* g, const orc_phase ph[2], double dt, int32_t relax_pressure,
                       double* alpha2, double* m1, double* m2, double* T1, double* T2, double* u,
                       double* v, double* w, double* E);
/* Pressure relaxation of one conservative state q[9] (order of
 * orc_hyperbolic's U: alpha1 rho1, alpha2 rho2, rho u, rho v, rho w,
 * alpha1 rho1 e1, alpha2 rho2 e2, rho E, alpha2), in place. */
void orc_pressure_relax_cell(const orc_phase ph[2], double* q);
/* cfl / max over cells and axes of (|u_d| + c)/h_d. */
double orc_hyperbolic_dt(const orc_grid* g, const orc_phase ph[2], double cfl, const double* alpha2,
                         const double* m1, const double* m2, const double* T1, const double* T2,
                         const double* u, const double* v, const double* w);

#ifdef __cplusplus
}
#endif
#endif
