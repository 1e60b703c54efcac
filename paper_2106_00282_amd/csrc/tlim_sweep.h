// Launchers of the LIM stages (eq. LIM).  One call advances up to `count`
// consecutive stages and returns how many it did (>= 1, equal to
// sweeps_per_launch(g, count)); the result is in `out`.  Several stages per
// launch are fused where the grid allows (temporal blocking), otherwise one
// stage is launched.  In FP64 the final stage (b = 0, flux form) may be among
// them: a launch with last = true ends the pass and, when Tit != NULL, also
// accumulates the pass reductions (dmax, tmax, bad) into ps.  The FP32
// correction form advances the float correction w = v - g (source
// qn = -tau A' g); its final stage is evaluated in double on g + w and the
// launch that reaches it writes out64 (rhs = g and rC in double) instead of
// out.
#pragma once

#include "tlim_internal.h"

namespace tlim {

// Parameters of consecutive stages (host arrays, already offset to the first
// stage of the launch): with lam == NULL stage k uses tau*b_k = tb[k];
// otherwise tau*b_k = tau * (*lam) * chat[k], lam pointing to device memory.
struct Stages {
    const double* lam;
    const double* tb;
    const double* chat;
};

// Number of stages the next launch will advance when `count` remain (the
// launches of a pass get equal shares of at most 8 or 10 stages, by tile height).
int sweeps_per_launch(const DevGrid& g, int count);

// The next Picard pass's coefficients, built by the launch that reaches the
// final stage when it can (blocked 2D launches): Lam = sum_k alpha_k
// lambda_k(T^(it+1)) and the Gershgorin bound (max into the row lam), with
// 1/C unchanged (equal p_inf); in the FP32 form the float conductivities and
// the correction source instead of Lam.  nc_done tells whether that
// happened.
struct NextCoef {
    double* lam;
    const double* alpha2;
    double* Lam;    // FP64 (must not be the Lam the pass reads)
    float* Lam32;   // FP32 correction form: float conductivities and the
    float* q32;     // correction source of the next pass (not the ones read)
    DevPhases ph;
    // partial densities: the Spitzer-Harm law reads rho = m1 + m2
    const double* m1;
    const double* m2;
    // FP64, last pass of a step: with next_step set the next step's first
    // coefficients instead -- the temperature relaxation of every cell from
    // (alpha2, T^{n+1}, T^{n+1}, m1, m2) as the relaxation kernel does it,
    // then Lambda and the bound at the relaxed state; the relaxed T and
    // alpha2 go to Tn and a2 (neither read by the pass).  1/C is the step's
    // (equal p_inf: it depends on the partial densities only).
    int next_step;
    double* Tn;
    double* a2;
    double eps;
};

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, Stages st, int count, bool last, double tau,
                    const double* Tit, PassSlots ps, const NextCoef* nc = nullptr, bool* nc_done = nullptr);

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* qn,
                    const float* Lam32, const float* rC32, float* out, Stages st, int count, bool last, double tau,
                    const double* rhs, const double* rC, double* out64, const double* Tit, PassSlots ps,
                    const NextCoef* nc = nullptr, bool* nc_done = nullptr, bool w_zero = false);

// One stage on a 3D grid by z-marching waves (tlim_sweep3d.hip): as
// launch_stage64 / launch_stage32, and with Tit != NULL also the pass
// reductions of launch_final64 (for the final stage pass sp.tb = 0).
bool use_z3d(const DevGrid& g);
template <typename R>
void launch_z3d(hipStream_t s, const DevGrid& g, int face, const R* v, const R* G, const R* Lam, const R* rC, R* out,
                StageParam sp, double tau, const double* Tit, PassSlots ps);
// Reverse stages of the adjoint on 3D grids by z-marching waves (arithmetic
// face means): psi_out = c_m (tb psi - tau rC A' psi) with the face gradient
// and dL/dg accumulated in place into gLam and dgpsi (psi = C^-1 lambda;
// launch_psi_from_lambda converts the first stage's input).
bool use_adj_z3d(const DevGrid& g, int face);
void launch_psi_from_lambda(hipStream_t s, int64_t n, const double* lam, const double* rC, double* psi);
void launch_adj_z3d(hipStream_t s, const DevGrid& g, const double* psi, const double* vprev, const double* Lam,
                    const double* rC, double* psi_out, double* dgpsi, double* gLam, double cm, double tb,
                    double tau);
// The first two float stages of an FP32 pass that starts from w = 0 on a 3D
// grid in one launch: stage 0 gives c_0 qn exactly, so the launch runs stage
// 1 on that input read from qn (sp0, sp1: the two stages' parameters).
void launch_z3d_two_from_zero32(hipStream_t s, const DevGrid& g, int face, const float* qn, const float* Lam32,
                                const float* rC32, float* out, StageParam sp0, StageParam sp1, double tau);
// The FP32 correction form's final stage on a 3D grid (as launch_final32).
void launch_z3d_final32(hipStream_t s, const DevGrid& g, int face, const float* w, const double* rhs,
                        const float* Lam32, const double* rC, double* out, double tau, const double* Tit,
                        PassSlots ps);

// Blocked FP64 stages that also keep their intermediate results: the result
// of the launch's stage k (k = 1 .. K-1) goes to stages + k*sstride and the
// last one to out.  Returns K, or -1 where blocking does not apply (then
// nothing is launched).
int launch_sweeps64_keep(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                         const double* Lam, const double* rC, double* out, Stages st, int count, double tau,
                         double* stages, int64_t sstride);

// Blocked reverse stages of the adjoint in the scaled form psi = C^-1 lambda
// (psi^(m-1) = c_m (tau b_m - tau A) psi^(m), the forward stage operator
// without source), for stages mt, mt-1, ..., mt-count+1 of one LIM pass:
//   psi_in   psi^(mt) (first = 1: lambda^(mt), scaled by 1/C on load)
//   stages   forward iterates, v^(j) at stages + j*sstride (j >= 1), v^(0) at v0
//   psi_out  psi^(mt-K)
//   dgpsi   += sum_m c_m psi^(m)           (dL/dg = C dgpsi)
//   gLam    += sum_m sum_f c_m tau w/2 (v_b - v_a)^(m-1) (psi_a - psi_b)^(m)
//             (dL/dLambda_cell through arithmetic face means)
// accumulate = 0 starts the sums at zero.  cm, tb: c_m and tau*b_m of the K
// stages in the order they are reversed.  When the launch reaches v^(0)
// (mt == K) and cell != NULL it finishes the pass as launch_adj_cell does
// (psi form) instead of writing psi_out, dgpsi and gLam.  Returns K, or -1
// where blocking does not apply (3D grid, harmonic faces): nothing is
// launched.
struct AdjCell {
    DevPhases ph;
    const double* Tit;     // T^(it), the lagged iterate of the pass
    const double* alpha2;
    const double *m1, *m2;  // partial densities (the Spitzer-Harm law reads rho = m1 + m2)
    double* acc;           // dL/dT^n accumulator
    double* mu;            // out: dL/dT^(it) through Lambda(T^(it))
    int init, first_pass;  // as launch_adj_cell
    double* k0a;           // accumulator rows of the dL/dk0 sums
    double* k0b;
};
int launch_adjoint_sweeps(hipStream_t s, const DevGrid& g, int face, const double* psi_in, int first,
                          const double* Lam, const double* rC, const double* stages, const double* v0,
                          int64_t sstride, int mt,
                          double* psi_out, double* dgpsi, double* gLam, int accumulate, const double* cm,
                          const double* tb, int count, double tau, const AdjCell* cell = nullptr);

}  // namespace tlim
