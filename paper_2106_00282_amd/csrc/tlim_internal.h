// Internal interface between the host runtime (tlim_runtime.cpp) and the
// gfx950 kernels (tlim_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlim {

// Grid as the kernels see it.  w[d] = scale_d / h_d^2 is the weight of a
// face normal to axis d (scale = 1 for heat, 4/3 on the own axis of a
// velocity component for the viscous sub-step).
struct DevGrid {
    int nx, ny, nz;
    int per[3];      // 1 = periodic axis
    double w[3];
    int64_t N;
};

// Material constants the kernels need (both phases).
struct DevPhases {
    double gamma[2], pinf[2], cv[2];
    double k0[2], T0[2], npow[2];
    double mu[2];
};

// Results of the per-pass reduction, read back to the host.
struct PassResult {
    double dmax;      // max |T^(it+1) - T^(it)|
    double tmax;      // max |T^(it+1)|
    double energy;    // sum (C1 T1 + C2 T2 + alpha_k p_inf,k), without the cell volume
    double bad;       // count of non-finite or T <= 0
    double lambda;    // Gershgorin bound of the next pass (when requested)
    double rr, gg;    // cycle mode: squared residual norm and squared |C g|
    double k0g[2];    // adjoint: dL/dk0 partial sums
};

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kPartialStride = 8;  // doubles per block in the partials array

// ---- launches (all enqueue on `s`, none synchronises) ----
void launch_relax(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double* alpha2,
                  const double* m1, const double* m2, double* T1, double* T2);

// Heat coefficients at (T, alpha2): Lam = sum alpha_k lambda_k(T), rC = 1/C_eff,
// rhs = Tn + tau rC (alpha1 I1 + alpha2 I2).  Optional float copies.
void launch_heat_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau,
                        const double* T, const double* alpha2, const double* m1, const double* m2,
                        const double* Tn, const double* src1, const double* src2, double* Lam,
                        double* rC, double* rhs, float* Lam32, float* rC32);

// Viscous coefficients: Lam = alpha1 mu1 + alpha2 mu2, rC = 1/(m1 + m2).
void launch_visc_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2,
                        const double* m1, const double* m2, double* Lam, double* rC, float* Lam32,
                        float* rC32);

// Gershgorin bound max_i 2 rC_i sum_f w Lam_f -> partials, then res->lambda.
void launch_gershgorin(hipStream_t s, const DevGrid& g, int face, const double* Lam, const double* rC,
                       double* partials, PassResult* res);

// Energy sum of the state -> res->energy.
void launch_energy(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2,
                   const double* m1, const double* m2, const double* T1, const double* T2,
                   double* partials, PassResult* res);

// One FP64 LIM stage: out = cm (rhs + tb v - tau rC sum_f w Lam_f (v_a - v_b)).
void launch_stage64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, double cm, double tb, double tau);
// Final FP64 stage (b = 0) in flux form: out = rhs + tau rC sum_f w Lam_f (v_b - v_a).
void launch_final64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, double tau);

// FP32 correction form, w = v - rhs:
//   q = -tau rC' D' rhs (computed in double, stored float), w0 = float(v0 - rhs)
//   w^(m) = cm (q + tb w - tau rC D w)                               (float)
//   out = rhs + tau rC64 sum_f w Lam'_f ((rhs+w)_b - (rhs+w)_a)        (double)
void launch_q32(hipStream_t s, const DevGrid& g, int face, const double* rhs, const double* v0,
                const float* Lam32, const float* rC32, double tau, float* q, float* w0);
void launch_stage32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* q,
                    const float* Lam32, const float* rC32, float* out, float cm, float tb, float tau);
void launch_final32(hipStream_t s, const DevGrid& g, int face, const float* w, const double* rhs,
                    const float* Lam32, const double* rC, double* out, double tau);

// After a pass: alpha2 update (B1 != 0) and reductions (dmax, tmax, bad).
void launch_pass_update(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps,
                        const double* Tit, const double* Tnew, const double* Tn, const double* alpha2n,
                        const double* alpha2it, const double* m1, const double* m2, double* alpha2out,
                        double* partials, PassResult* res);

// Cycle mode: relative BE residual || C(rhs - v) - tau D v ||^2, || C rhs ||^2 -> res->rr, gg.
void launch_be_residual(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                        const double* Lam, const double* rC, double tau, double* partials, PassResult* res);

// Adjoint of one stage (FP64):
//   dg += cm lam;  gLam_a += sum_f cm tau w (v_b - v_a)(lam_a rC_a - lam_b rC_b) dLam_f/dLam_a;
//   lam_out = cm (tb lam + tau sum_f w Lam_f (lam_b rC_b - lam_a rC_a)).
void launch_adj_stage(hipStream_t s, const DevGrid& g, int face, const double* lam, const double* vprev,
                      const double* Lam, const double* rC, double* lam_out, double* dg, double* gLam,
                      double cm, double tb, double tau);
// After a reversed pass: acc += dg + lam0; mu = gLam dLam/dT(Tit); k0 partial sums;
// if first_pass: acc += mu.
void launch_adj_cell(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* Tit,
                     const double* alpha2, const double* gLam, const double* dg, const double* lam0,
                     double* acc, double* mu, int first_pass, double* partials, PassResult* res);

void launch_fill(hipStream_t s, double* p, double v, int64_t n);
void launch_copy(hipStream_t s, double* dst, const double* src, int64_t n);

}  // namespace tlim
