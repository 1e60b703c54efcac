/*
 * tlim — parabolic sub-step (heat conduction + viscosity) of the
 * two-temperature diffuse-interface model of Zhang, Menshov, Wang and Shen,
 * "Diffuse interface relaxation model for two-phase compressible flows with
 * diffusion processes" (arXiv 2106.00282), on one AMD Instinct MI355X
 * (gfx950).
 *
 * One call of tlim_advance_parabolic is one parabolic step of the paper's splitting
 * (Sec. 3): the viscous part (Sec. 3.2, eq. viscous), instantaneous
 * temperature relaxation in interface cells (Sec. 3.4.1) and heat conduction
 * (Sec. 3.4.2, Algorithm 1).  Both diffusion problems are advanced with the
 * method of local iterations with Chebyshev parameters (Sec. 3.2, eqs. LIM
 * and LIM_last): 2P-1 explicit stencil sweeps,
 * P = ceil(pi/4 sqrt(tau lambda_max + 1)), the last one in conservative
 * flux form.  Heat conduction wraps the sweeps in a Picard loop with face
 * conductivities lagged at the previous iterate (Algorithm 1).
 * tlim_advance_hyperbolic runs the mechanical stage that comes before it in
 * the splitting: the hyperbolic part (Sec. 3.1) and the pressure relaxation
 * (Sec. 3.3).
 *
 * ---------------------------------------------------------------- conventions
 * Memory.  Every pointer argument named *_dev is a device pointer on the
 * device that was current at tlim_create; every other pointer is host
 * memory.  The caller owns all memory, including the workspace it binds with
 * tlim_bind_workspace; the library only borrows pointers during a call and
 * never frees caller memory.  Fields are dense arrays of nx*ny*nz values
 * in C order with x fastest, index i + nx*(j + ny*k); the context keeps its
 * state in float64, and tlim_set_field / tlim_get_field also take float32.
 * Streams.  All device work of a context is enqueued on the HIP stream given
 * to tlim_create (NULL = the null stream).  Calls that return values
 * computed on the device (spectral bound, step report, adjoint k0
 * gradient, hyperbolic time step and report) synchronise that stream before
 * returning; tlim_set_field and tlim_get_field do not.
 * Errors.  Every entry point returns a tlim_status; nothing is thrown across
 * the ABI.  TLIM_E_ARG leaves the context unchanged.  tlim_last_error gives
 * a message for the last failing call on a context.
 * Threading.  Contexts are independent; a context must not be used from two
 * threads at once.
 */
#ifndef TLIM_H
#define TLIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLIM_OK = 0,
    TLIM_E_ARG = 1,      /* invalid argument; nothing was changed */
    TLIM_E_STATE = 2,    /* missing phase, field or workspace */
    TLIM_E_HIP = 3,      /* a HIP runtime call failed */
    TLIM_E_NOMEM = 4,    /* bound workspace smaller than required */
    TLIM_E_NOCONV = 5,   /* Picard or cycle tolerance not met; fields hold the last iterate */
    TLIM_E_NUMERIC = 6   /* non-finite or non-positive temperature found after a pass */
} tlim_status;

enum { TLIM_PERIODIC = 0, TLIM_ADIABATIC = 1 };         /* boundary per axis */
enum { TLIM_FP64 = 0, TLIM_FP32 = 1 };                 /* arithmetic of the sweeps */
enum { TLIM_DTYPE_F64 = 0, TLIM_DTYPE_F32 = 1 };       /* element type of a caller's field buffer */
enum { TLIM_ORDER_INTERLEAVED = 0, TLIM_ORDER_PAPER = 1, TLIM_ORDER_ASCENDING = 2 };
enum { TLIM_FACE_ARITH = 0, TLIM_FACE_HARMONIC = 1 };
/* whole_step: AUTO uses the one-launch step for the steps whose P would
 * otherwise be read back pass by pass: while the context has no schedule
 * history for the step's pass count, or one that has not yet held for a
 * step (a step is predicted only after that); ALWAYS for every eligible
 * step, NEVER for none. */
enum { TLIM_WHOLE_AUTO = 0, TLIM_WHOLE_ALWAYS = 1, TLIM_WHOLE_NEVER = 2 };

/* Fields of the state (Sec. 3.4, data of Algorithm 1): volume fraction of
 * phase 2, partial densities m_k = alpha_k rho_k (constant in this step),
 * phase temperatures, velocity components, external heat sources I_k, and
 * the mixture total energy density rho E (optional).  Once E has been set,
 * every step updates it as the six-equation model's mixture energy equation
 * does in this sub-step: the viscous part adds, per velocity component, the
 * divergence of the work of the viscous flux, tau sum_f w_f mu_f uh_f
 * (uh_b - uh_a) with the predicted velocity uh (Sec. 3.2, total-energy
 * update); the heat part adds C_eff (T^{n+1} - T^n) with the last Picard
 * pass's C_eff and the relaxed T^n, which is that pass's conductive flux
 * divergence plus tau sum_k alpha_k I_k (Sec. 3.4.2, heat-conduction
 * system).  Steps with E set are not pipelined. */
typedef enum {
    TLIM_ALPHA2 = 0, TLIM_M1 = 1, TLIM_M2 = 2, TLIM_T1 = 3, TLIM_T2 = 4,
    TLIM_U = 5, TLIM_V = 6, TLIM_W = 7, TLIM_SRC1 = 8, TLIM_SRC2 = 9,
    TLIM_E = 10,
    TLIM_NFIELDS = 11
} tlim_field;

/* Cell-centred grid: n[0] cells along x, n[1] along y, n[2] along z (1 for
 * unused axes), spacings h, boundary condition per axis. */
typedef struct {
    int64_t n[3];
    double h[3];
    int32_t bc[3];
} tlim_grid;

/* Conductivity laws of a phase. */
enum {
    TLIM_LAW_POWER = 0,   /* lambda(T) = k0 (T/T0)^npow (Sec. 3.4.2 allows lambda = lambda(T)) */
    TLIM_LAW_SPITZER = 1  /* lambda(rho, T) = k0 (T/T0)^npow / ln Lambda_ei(rho, T): the
                             Spitzer-Harm form of Sec. 4.4 (npow = 5/2 there; the prefactor,
                             charge state and atomic number go into k0) */
};

/* One phase: stiffened-gas EOS (eqs. eos_stiffened, eos_stiffened2:
 * gamma, p_inf, C_v, q), conductivity law, dynamic viscosity mu (Sec. 3.2).
 *
 * law = TLIM_LAW_SPITZER takes the Coulomb logarithm of Sec. 4.4,
 *   ln Lambda_ei = max(1, ln(l_D / l_LD))  if l_LD >= l_dB,
 *                  max(1, ln(l_D / l_dB))  otherwise,
 * with the Debye, Landau and de Broglie lengths written as
 *   l_D = sh_D sqrt(T / rho),  l_LD = sh_LD / T,  l_dB = sh_dB / sqrt(T),
 * rho the cell's mixture density m1 + m2.  The constants sh_* carry the
 * physical constants, charge state and atomic number in the caller's
 * units (sh_D > 0, sh_LD >= 0, sh_dB >= 0, not both zero).  They are
 * ignored under TLIM_LAW_POWER. */
typedef struct {
    double gamma, pinf, cv, q;
    double k0, T0, npow;
    double mu;
    int32_t law;                /* TLIM_LAW_* */
    double sh_D, sh_LD, sh_dB;  /* Spitzer-Harm length constants */
} tlim_phase;

/* Options of one parabolic step. */
typedef struct {
    double dt;                   /* time step tau > 0 */
    int32_t passes;              /* Picard passes (maximum when picard_tol > 0), 1..64 */
    double picard_tol;           /* stop when max|T^(it+1)-T^(it)|/max|T^(it+1)| < tol; 0 = run all */
    int32_t order;               /* TLIM_ORDER_*: order of the 2P-2 inner Chebyshev parameters */
    int32_t face_mean;           /* TLIM_FACE_*: face value of the cell conductivities */
    int32_t cycle_mode;          /* 1: Chebyshev-Richardson cycles to the backward-Euler solution */
    double cycle_tol;            /* cycle mode: relative residual target */
    int32_t max_cycles;          /* cycle mode: cycle limit per pass */
    double alpha_eps;            /* interface (mixed) cell: eps < alpha2 < 1 - eps */
    int32_t do_viscous;          /* run the viscous sub-step first (needs U[,V[,W]]) */
    const double* frozen_lambda; /* nullable, `passes` entries: lambda_max per pass instead of Gershgorin */
    const double* frozen_visc;   /* nullable, 3 entries: lambda_max per velocity component */
    int32_t time_sweeps;         /* 1: time the sweep launches with HIP events (report.sweep_ms) */
    int32_t visc_heating;        /* with do_viscous: the viscous part also heats the phases (Sec. 3.2,
                                    phase internal-energy update with the predicted velocity) */
    int32_t whole_step;          /* TLIM_WHOLE_*: when an FP64 2D step without sources and with equal
                                    p_inf, whose tiles all fit on the device at once, runs as one
                                    cooperative launch (relaxation and every pass, P decided on the
                                    device from the reduced lambda_G, no host prediction) instead of
                                    one launch per block of stages.  Same results up to rounding
                                    order.  Its grid barriers wait a bounded time (about a second;
                                    the environment variable TLIM_STEP2D_SPIN_LIMIT, read at
                                    tlim_create, sets the poll count, a test hook); a wait that runs
                                    out makes the step return TLIM_E_HIP (or the call that verifies
                                    a pipelined one) with alpha2, T1 and T2 marked as not set, so
                                    that the next step returns TLIM_E_STATE until they are set
                                    again */
} tlim_step_opts;

#define TLIM_MAX_PASSES 64
/* Per-step report, filled when a non-NULL pointer is passed. */
typedef struct {
    int32_t passes_run;
    int32_t converged;
    int32_t P[TLIM_MAX_PASSES];           /* Chebyshev parameter count per pass */
    double lambda_G[TLIM_MAX_PASSES];     /* lambda_max used per pass */
    double err[TLIM_MAX_PASSES];          /* Picard change per pass (Algorithm 1) */
    int32_t cycles[TLIM_MAX_PASSES];      /* cycle mode: cycles per pass */
    double residual[TLIM_MAX_PASSES];     /* cycle mode: final relative residual per pass */
    int32_t visc_P[3];
    double visc_lambda_G[3];
    double energy_before, energy_after;   /* sum_i vol (sum_k C_k T_k + alpha_k p_inf,k) */
    int64_t sweeps;                       /* stencil sweeps run (heat + viscous) */
    int64_t sweep_launches;               /* sweep kernel launches (<= sweeps when fused) */
    double sweep_ms;                      /* time_sweeps: summed event time of the sweep launches
                                             enqueued behind earlier device work of the step (a pass
                                             enqueued right after a readback is left out: its events
                                             would also time the host's enqueueing) */
    int64_t bad_cells;                    /* cells with non-finite or T <= 0 after the last pass */
    int32_t predicted;                    /* 1: P of every pass was predicted from the previous step
                                             and confirmed (no per-pass readback) */
    int32_t mispredicted;                 /* 1: a predicted P was wrong; the heat passes were rerun
                                             with one readback per pass (sweeps counts the rerun only) */
    int64_t pipelined_steps;              /* context totals so far: steps run pipelined (see */
    int64_t pipeline_redos;               /* tlim_advance_parabolic) and pipelined steps redone */
    int64_t timed_sweeps;                 /* time_sweeps: the stages and launches sweep_ms covers */
    int64_t timed_launches;
} tlim_step_report;

typedef struct tlim_ctx tlim_ctx;

/* Create a context for one grid.  precision = TLIM_FP64 or TLIM_FP32 (the
 * FP32 form: stencil sweeps in float, state, energy, residual and Picard
 * sums, relaxation and lambda_max in double).  hip_stream: hipStream_t or
 * NULL.  Errors: TLIM_E_ARG for n < 1, h <= 0, an unknown bc or precision;
 * TLIM_E_HIP if the device cannot be queried. */
tlim_status tlim_create(const tlim_grid* grid, int32_t precision, void* hip_stream, tlim_ctx** out);

/* Release a context (not the caller's memory).  NULL is accepted. */
tlim_status tlim_destroy(tlim_ctx* ctx);

/* Device workspace the context needs for state and stepping, in bytes. */
tlim_status tlim_workspace_bytes(const tlim_ctx* ctx, size_t* bytes);

/* Bind caller-allocated device memory (256-byte aligned, at least
 * tlim_workspace_bytes) as the context's workspace.  Fields set before a
 * new binding are lost.  Errors: TLIM_E_NOMEM if too small, TLIM_E_ARG if
 * misaligned or NULL. */
tlim_status tlim_bind_workspace(tlim_ctx* ctx, void* dev_ptr, size_t bytes);

/* Set phase k (0 or 1).  Errors: TLIM_E_ARG for k out of range, gamma <= 1,
 * cv <= 0, k0 < 0, T0 <= 0, mu < 0, an unknown law, or Spitzer-Harm
 * constants outside the ranges above. */
tlim_status tlim_set_phase(tlim_ctx* ctx, int32_t k, const tlim_phase* phase);

/* Copy a field (Sec. 3.4, the data of Algorithm 1) from caller device
 * memory into the context: nx*ny*nz values in the layout of the conventions,
 * of type dtype (TLIM_DTYPE_F64, or TLIM_DTYPE_F32, widened to the state's
 * float64 on the device).  Sources are optional (absent = 0); velocity is
 * needed only for the viscous sub-step.  Errors: TLIM_E_ARG for an unknown
 * field or dtype or a NULL pointer (nothing changed), TLIM_E_STATE without a
 * workspace. */
tlim_status tlim_set_field(tlim_ctx* ctx, int32_t field, const void* src_dev, int32_t dtype);

/* Copy a field out of the context into caller device memory of type dtype
 * (float64, or rounded to float32 on the device); a pending pipelined step
 * is completed first (see tlim_advance_parabolic).  Errors: TLIM_E_ARG as
 * for tlim_set_field, TLIM_E_STATE for a field that is not set. */
tlim_status tlim_get_field(tlim_ctx* ctx, int32_t field, void* dst_dev, int32_t dtype);

/* Mark an optional field (TLIM_U, TLIM_V, TLIM_W, TLIM_SRC1, TLIM_SRC2,
 * TLIM_E) as not set: absent sources are zero again and the total energy is
 * no longer updated.  Errors: TLIM_E_ARG for any other field. */
tlim_status tlim_clear_field(tlim_ctx* ctx, int32_t field);

/* Gershgorin bound lambda_G = max_i 2 d_i of the heat operator A = C^-1 D
 * (Sec. 3.2 needs lambda_max of L_h; D from eq. qk_dis) for the current
 * fields after temperature relaxation; the fields themselves are not
 * changed.  The explicit stability limit is 2 / lambda_G.  Synchronises. */
tlim_status tlim_spectral_bound(tlim_ctx* ctx, int32_t face_mean, double alpha_eps, double* lambda_out);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc): the value tlim_spectral_bound
 * returns, with no context, no workspace and no allocation of any kind.
 * Inputs are the caller's device fields alpha2, m1, m2, T1, T2 (dense
 * float64, layout of the conventions) on the grid `grid` with the two
 * phases `phases` (checked as tlim_create and tlim_set_phase check them);
 * the bound is written to lambda_dev[0] (device memory) on hip_stream (NULL
 * = the null stream) and nothing synchronises.  The current device must be
 * the one that holds the fields.
 * Scratch: a library-owned device array of 256 doubles (2 KiB) per device,
 * held until the process ends; every call clears it first with a kernel.
 * Calls that overlap on one device race on it.  Limit: at most 2^31 - 1
 * cells (larger grids return TLIM_E_ARG).  Errors: TLIM_E_ARG (nothing
 * launched), TLIM_E_HIP; tlim_last_error(NULL) gives the reason of the
 * calling thread's last failing call. */
tlim_status tlim_spectral_bound_noalloc(const tlim_grid* grid, const tlim_phase phases[2], int32_t face_mean,
                                        double alpha_eps, const double* alpha2_dev, const double* m1_dev,
                                        const double* m2_dev, const double* T1_dev, const double* T2_dev,
                                        double* lambda_dev, void* hip_stream);

/* Advance the fields by one parabolic step: viscous part (optional),
 * temperature relaxation, Picard loop of LIM passes (Algorithm 1).
 * report may be NULL.  Returns TLIM_E_NOCONV when picard_tol > 0 (or the
 * cycle tolerance) was not met, TLIM_E_NUMERIC when a non-finite or
 * non-positive temperature appears; in both cases the fields hold the last
 * iterate.  The number of sweeps of a pass, 2P-1, follows from lambda_max of
 * that pass.  With frozen_lambda the host knows it; otherwise, when the
 * previous step ran the same number of passes (and picard_tol = 0, no cycle
 * mode), P of every pass is predicted from that step, the stages read
 * lambda_max from device memory, and one readback at the end confirms the
 * predictions (a wrong one rolls the heat part back and reruns it with one
 * readback per pass).  Otherwise it synchronises once per Picard pass.
 *
 * Pipelining.  A predicted step with report == NULL, no viscous part, no
 * timing, equal p_inf, on a 2D grid without sources, returns as soon as it
 * is enqueued; its readback is checked by the next call on the context,
 * after that call has enqueued its own step, so consecutive steps run back
 * to back on the device.  A wrong prediction found then redoes the checked
 * step (and reruns the newer one with its own readback); a non-finite or
 * non-positive temperature of the checked step is returned by that call as
 * TLIM_E_NUMERIC.  Every other entry point, and tlim_finish, completes the
 * pending step first. */
tlim_status tlim_advance_parabolic(tlim_ctx* ctx, const tlim_step_opts* opts, tlim_step_report* report);

/* Complete a pending pipelined step (see tlim_advance_parabolic): wait for its
 * readback, redo it if its schedule was mispredicted, and return its status
 * (TLIM_OK when nothing is pending).  Synchronises. */
tlim_status tlim_finish(tlim_ctx* ctx);

/* Forward run of nsteps heat steps with checkpoints for the adjoint: T^n is
 * copied to ckpt_dev + (n / ckpt_every) * N before every step n with
 * n % ckpt_every == 0 (so ckpt_dev holds ceil(nsteps/ckpt_every) fields),
 * and lambda_max of every pass goes to lam_out[n * passes + it] (host).
 * Requires equal p_inf of the two phases, no sources, no viscous part, no
 * cycle mode, picard_tol = 0.  Relaxation is applied by tlim_advance_parabolic as usual. */
tlim_status tlim_forward_checkpointed(tlim_ctx* ctx, const tlim_step_opts* opts, int32_t nsteps,
                                      int32_t ckpt_every, double* ckpt_dev, double* lam_out);

/* Device scratch tlim_adjoint_parabolic needs for nsteps steps of the frozen
 * schedule lam (nsteps*passes host values, as written by
 * tlim_forward_checkpointed): every stage iterate of one step's passes, whose
 * count follows from the largest P = ceil(pi/4 sqrt(dt lam + 1)) of the
 * schedule (Sec. 3.2, eq. LIM).  Errors: TLIM_E_ARG for NULL pointers,
 * nsteps < 1, passes out of range, dt not finite and > 0, or a schedule
 * entry that is negative or not finite. */
tlim_status tlim_adjoint_workspace_bytes(const tlim_ctx* ctx, const tlim_step_opts* opts, int32_t nsteps,
                                         const double* lam, size_t* bytes);

/* Device scratch with which tlim_adjoint_parabolic keeps every step of a
 * checkpoint interval (min(ckpt_every, nsteps) step blocks of the size above,
 * plus the shared adjoint fields): each interval is then recomputed once, and
 * no step twice.  Same results, bit for bit, as with the smaller workspace;
 * the adjoint takes whichever layout adj_ws_bytes holds.  Errors as
 * tlim_adjoint_workspace_bytes, and TLIM_E_ARG for ckpt_every < 1. */
tlim_status tlim_adjoint_workspace_bytes_kept(const tlim_ctx* ctx, const tlim_step_opts* opts, int32_t nsteps,
                                              int32_t ckpt_every, const double* lam, size_t* bytes);

/* Discrete adjoint of nsteps heat steps with the frozen schedule lam
 * (nsteps*passes host values, as written by tlim_forward_checkpointed):
 * given dL/dT^N (dL_dTN_dev), returns dL/dT^0 (dL_dT0_dev, device) and
 * dL/dk0 of both phases (dL_dk0, 2 host doubles).  Each step is recomputed
 * from the nearest checkpoint, keeping every stage iterate in adj_ws_dev
 * (with a workspace of tlim_adjoint_workspace_bytes_kept bytes, every step of
 * the interval at once, so that no step is recomputed twice), and
 * reversed stage by stage (lambda^(m-1) = c_m (tau b_m lambda^(m) -
 * tau D C^-1 lambda^(m)), with the face-conductivity gradient chained
 * through Lambda(T^(it)) of every Picard pass).  The forward model is the
 * heat step without relaxation, which is the identity on the equilibrium
 * states the forward run produces.  Same restrictions as
 * tlim_forward_checkpointed.  The recomputation and the reverse stages run
 * in FP64 also in FP32 contexts: the result is the gradient of the FP64
 * discretisation at the checkpointed states.  Synchronises. */
tlim_status tlim_adjoint_parabolic(tlim_ctx* ctx, const tlim_step_opts* opts, int32_t nsteps, int32_t ckpt_every,
                         const double* ckpt_dev, const double* lam, const double* dL_dTN_dev,
                         double* dL_dT0_dev, double* dL_dk0, void* adj_ws_dev, size_t adj_ws_bytes);

/* ---- Hyperbolic part and pressure relaxation (the mechanical stage on the
 * other side of the splitting, Sec. 3.1 and Sec. 3.3) ---- */

typedef struct {
    double dt;               /* time step > 0; stable for dt * (|u_d| + c) / h_d <= 1 on every axis */
    int32_t relax_pressure;  /* 1: pressure relaxation after each directional sweep */
} tlim_hyp_opts;

typedef struct {
    double bad_cells;        /* cells that left 0 < alpha2 < 1 or lost a positive temperature */
} tlim_hyp_report;

/* One step of the hyperbolic part of the six-equation model: the Godunov
 * method with HLLC faces on eq. vectorForm (the phase masses, momentum,
 * total energy and alpha_2, and the non-conservative phase internal-energy
 * equations with R(U) du/dx), one directional sweep per axis with more than
 * one cell in the order x, y, z (dimensional splitting), each followed by
 * the pressure relaxation of Sec. 3.3 when opts->relax_pressure is set:
 * step 1 relaxes alpha_k at fixed phase masses with d(alpha_k rho_k e_k) =
 * -p d alpha_k up to the pressure that saturates alpha_1 + alpha_2 = 1,
 * step 2 takes the pressure of the mixture at the total energy, step 3 the
 * phase energies at that pressure.  HLLC details that the paper leaves open:
 * Davis wave speeds, the model's sound speed c^2 = Y_1 c_1^2 + Y_2 c_2^2,
 * star states that scale every advected density (phase masses, tangential
 * momenta, phase internal energies) by (S_K - u_K)/(S_K - S*).  An adiabatic
 * axis is a reflecting wall.
 *
 * Reads and writes the state: alpha2, M1, M2, T1, T2 (from the phase
 * internal energies by eq. eos_stiffened2), the velocity U, V, W and E
 * (rho E).  Velocity components and E that are not set count as zero and as
 * the energy of the state, and are set afterwards.  Every cell must hold
 * both phases (0 < alpha2 < 1, M1 > 0, M2 > 0).  The step runs in FP64 in
 * both precisions, uses the heat step's scratch arrays and cancels its
 * prepared start.  With report != NULL it synchronises and returns
 * TLIM_E_NUMERIC if a cell left the admissible range (the fields then hold
 * the offending values).  Errors: TLIM_E_ARG (dt not finite or <= 0),
 * TLIM_E_STATE (workspace, phases or the five state fields missing). */
tlim_status tlim_advance_hyperbolic(tlim_ctx* ctx, const tlim_hyp_opts* opts, tlim_hyp_report* report);

/* The largest stable time step of the hyperbolic part scaled by cfl:
 * cfl / max over cells and axes with more than one cell of (|u_d| + c)/h_d
 * (0 if no axis has more than one cell).  Synchronises.  Errors: TLIM_E_ARG
 * (cfl not finite or <= 0, NULL dt_out), TLIM_E_STATE. */
tlim_status tlim_hyperbolic_dt(tlim_ctx* ctx, double cfl, double* dt_out);

/* Human-readable name of a status, and the last error message of a context
 * (with NULL: of the calling thread's last failing context-free call). */
const char* tlim_status_str(tlim_status s);
const char* tlim_last_error(const tlim_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
