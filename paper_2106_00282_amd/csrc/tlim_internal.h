// Internal interface between the host runtime (tlim_runtime.cpp) and the
// gfx950 kernels (tlim_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tlim.h"

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
    double gamma[2], pinf[2], cv[2], qf[2];  // SG EOS (qf: the constant q of eq. eos_stiffened)
    double k0[2], T0[2], invT0[2], npow[2];
    double mu[2];
    // sh_law[k] = 1: phase k follows the Spitzer-Harm law (else the power
    // law); spitzer = either phase does; logarithms of its length constants
    int sh_law[2], spitzer;
    double ln_shD[2], ln_shLD[2], ln_shdB[2];
};

constexpr int kMaxPasses = 64;

// Reductions.  Every reduction result ("target") owns a row of kSlots
// doubles in the accumulator array; a block folds its cells and adds one
// atomic to slot (block % kSlots) of the row -- atomicMax on the bit pattern
// for non-negative maxima (exact, order-independent), atomicAdd for sums --
// so no address sees more than blocks/kSlots atomics.  Kernels that need a
// result on the device fold the row themselves (row_max); launch_collect
// folds rows into one double each for the host readback.
constexpr int kSlots = 256;
enum {
    kTgtPass = 0,  // 4 targets per Picard pass: lambda_G, dmax, tmax, bad
    kTgtLambda = 4 * kMaxPasses,
    kTgtEnergy,
    kTgtRR,
    kTgtGG,
    kTgtK0a,
    kTgtK0b,
    kTgtFlag,      // whole-step kernel: failure count (schedule out of range, barrier time-out)
    kTgtNextStep,  // bound of the next step's first pass, built by this step's last launch
    kTgtHypBad,    // hyperbolic step: cells that left 0 < alpha2 < 1 or lost a positive T
    kTgtHypRate,   // hyperbolic step: max (|u_d| + c)/h_d
    kTgtVisc,      // viscous part: bound of velocity component c in row kTgtVisc + c
    kTgtVisc1,
    kTgtVisc2,
    kTgtP0,        // whole-step kernel: P of pass it in slot 0 of row kTgtP0 + it
    kTargets = kTgtP0 + kMaxPasses
};
__host__ __device__ constexpr int tgt_lam(int it) { return 4 * it; }
__host__ __device__ constexpr int tgt_dmax(int it) { return 4 * it + 1; }
__host__ __device__ constexpr int tgt_tmax(int it) { return 4 * it + 2; }
__host__ __device__ constexpr int tgt_bad(int it) { return 4 * it + 3; }
// reduction of a target: sums for counts and sums, max otherwise
__host__ __device__ constexpr bool tgt_is_sum(int t) {
    return (t < kTgtLambda && (t & 3) == 3) || t == kTgtEnergy || t == kTgtRR || t == kTgtGG || t == kTgtK0a ||
           t == kTgtK0b || t == kTgtFlag || t == kTgtHypBad;
}

// Results folded for the host (one double per target).
struct PassResult {
    double v[kTargets];
    // sequence number of the fold that wrote v (pipelined steps): published
    // after every value, so a host that reads it sees the values
    unsigned long long seq;
};

// Fold rows [t0, t1) of the accumulator into res->v[t0..t1) (res may be
// pinned host memory); consume = 1 also zeroes the rows.  move_from >= 0:
// afterwards row t0 takes the contents of row move_from, which is zeroed.
// seq != 0: the last workgroup to finish then stores seq into res->seq with
// a system-scope release, counting the workgroups in *done (zero before the
// launch, zero again after it).
void launch_collect(hipStream_t s, double* acc, PassResult* res, int t0, int t1, int consume, int move_from = -1,
                    unsigned long long seq = 0, unsigned* done = nullptr);
// Zero rows [t0, t1) of the accumulator.
void launch_zero_rows(hipStream_t s, double* acc, int t0, int t1);

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

// Rows of the pass reductions of one Picard pass.
struct PassSlots {
    double* dmax;  // nullable: the Picard change max |T^(it+1) - T^(it)| is then not formed
    double* tmax;
    double* bad;
};

// ---- launches (all enqueue on `s`, none synchronises) ----
// Relaxation in place; also writes the relaxed T to Tn and alpha2 to a2n (each nullable).
void launch_relax(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double* alpha2,
                  const double* m1, const double* m2, double* T1, double* T2, double* Tn, double* a2n);

// Heat coefficients at (T, alpha2): Lam = sum alpha_k lambda_k(T), rC = 1/C_eff,
// rhs = Tn + tau rC (alpha1 I1 + alpha2 I2).  rC and rhs may be NULL (not
// written).  Optional float copies.
void launch_heat_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau,
                        const double* T, const double* alpha2, const double* m1, const double* m2,
                        const double* Tn, const double* src1, const double* src2, double* Lam,
                        double* rC, double* rhs, float* Lam32, float* rC32);

// Viscous coefficients: Lam = alpha1 mu1 + alpha2 mu2, rC = 1/(m1 + m2).
void launch_visc_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2,
                        const double* m1, const double* m2, double* Lam, double* rC, float* Lam32,
                        float* rC32);

// Heat coefficients plus the Gershgorin bound (max into the accumulator row
// lam) in one stencil pass over (T, alpha2).  With q32 != NULL (FP32
// contexts) also the correction-form source and start: q32 = -tau rC' D' g,
// w0 = float(Tn - g).
void launch_heat_coeffs_bound(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                              const double* T, const double* alpha2, const double* m1, const double* m2,
                              const double* Tn, const double* src1, const double* src2, double* Lam, double* rC,
                              double* rhs, float* Lam32, float* rC32, float* q32, float* w0, double* lam);

// 2D grids (nz == 1) without sources: the same coefficients and bound from
// one pass over (T, alpha2) in column strips.  g = Tn is not copied (the
// stages read Tn).  rebuild = 0 keeps rC (and rC32) from an earlier pass of
// the step -- valid when 1/C does not depend on T (equal p_inf).  Lam may be
// NULL (FP32 contexts need Lam32 only); q32 as above; w0 = 0 is written
// only when w0 != NULL.
// With T2_relax != NULL the kernel first relaxes every cell from (alpha2,
// T = T1, T2_relax, m1, m2) -- as launch_relax -- and builds the coefficients
// at the relaxed state (rebuild implied); the relaxed T goes to Tn_out (also
// g, so Tn is not read), the relaxed alpha2 to a2_out (alpha2 itself is not
// written).
bool coeffs2d_applies(const DevGrid& g);
void launch_coeffs2d(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                     const double* T, const double* alpha2, const double* m1, const double* m2, const double* Tn,
                     int rebuild, double* Lam, double* rC, float* Lam32, float* rC32, float* q32, float* w0,
                     double* lam, const double* T2_relax = nullptr, double* Tn_out = nullptr,
                     double* a2_out = nullptr);

// Gershgorin bound max_i 2 rC_i sum_f w Lam_f -> max into the row lam.
// The Gershgorin bounds of the three velocity components of the viscous part
// in one pass over (Lambda, 1/C): component c with the face weights wc[c]
// (its axis scaled by 4/3), into rows + c*kSlots, for the components with
// bit c of mask set.
void launch_gershgorin_visc(hipStream_t s, const DevGrid& g, int face, const double* Lam, const double* rC,
                            const double wc[3][3], int mask, double* rows);

// Energy sum of the state -> added to the row energy.
void launch_energy(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2,
                   const double* m1, const double* m2, const double* T1, const double* T2, double* energy);

// Stage parameter of a LIM stage: tau*b either given (lam == NULL: tb) or
// taken from the device-resident bound, tau * row_max(lam) * chat, lam being
// the accumulator row of the pass's lambda_G.
struct StageParam {
    const double* lam;
    double tb;
    double chat;
};

// One FP64 LIM stage: out = cm (rhs + tb v - tau rC sum_f w Lam_f (v_a - v_b)), cm = 1/(1+tb).
void launch_stage64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, StageParam sp, double tau);
// Final FP64 stage (b = 0) in flux form: out = rhs + tau rC sum_f w Lam_f (v_b - v_a).
// With Tit != NULL it also accumulates the pass reductions into ps.
void launch_final64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, double tau, const double* Tit, PassSlots ps);

// FP32 correction form, w = v - rhs:
//   q = -tau rC' D' rhs (computed in double, stored float), w0 = float(v0 - rhs)
//   w^(m) = cm (q + tb w - tau rC D w)                               (float)
//   out = rhs + tau rC64 sum_f w Lam'_f ((rhs+w)_b - (rhs+w)_a)        (double)
void launch_q32(hipStream_t s, const DevGrid& g, int face, const double* rhs, const double* v0,
                const float* Lam32, const float* rC32, double tau, float* q, float* w0);
void launch_stage32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* q,
                    const float* Lam32, const float* rC32, float* out, StageParam sp, double tau);
void launch_final32(hipStream_t s, const DevGrid& g, int face, const float* w, const double* rhs,
                    const float* Lam32, const double* rC, double* out, double tau, const double* Tit, PassSlots ps);

// After a pass: alpha2 update (B1 != 0) and the pass reductions into ps.
void launch_pass_update(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps,
                        const double* Tit, const double* Tnew, const double* Tn, const double* alpha2n,
                        const double* alpha2it, const double* m1, const double* m2, double* alpha2out,
                        PassSlots ps);

// Cycle mode: || C(rhs - v) - tau D v ||^2 and || C rhs ||^2 added to the rows rr, gg.
void launch_be_residual(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                        const double* Lam, const double* rC, double tau, double* rr, double* gg);

// Adjoint of one stage (FP64):
//   dg += cm lam;  gLam_a += sum_f cm tau w (v_b - v_a)(lam_a rC_a - lam_b rC_b) dLam_f/dLam_a;
//   lam_out = cm (tb lam + tau sum_f w Lam_f (lam_b rC_b - lam_a rC_a)).
void launch_adj_stage(hipStream_t s, const DevGrid& g, int face, const double* lam, const double* vprev,
                      const double* Lam, const double* rC, double* lam_out, double* dg, double* gLam,
                      double cm, double tb, double tau);
// After a reversed pass: acc += dg + lam0 (with rCpsi != NULL the two are in
// psi = C^-1 lambda form and divided by rCpsi = 1/C first; init = 1 starts
// acc at zero instead of reading it); mu = gLam dLam/dT(Tit); the two dL/dk0
// sums are added to the rows k0a, k0b; if first_pass: acc += mu.
// Hyperbolic part (tlim_hyperbolic.hip).  Component arrays in the order
// alpha_1 rho_1, alpha_2 rho_2, rho u, rho v, rho w, alpha_1 rho_1 e_1,
// alpha_2 rho_2 e_2, rho E, alpha_2; the primitive fields in the matching
// order m1, m2, u, v, w, T1, T2, rho E, alpha2 (u, v, w, rho E may be NULL
// on input: zero, and the energy of the state).
void launch_hyp_cons(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* const prim[9],
                     double* const U[9]);
// One Godunov sweep along axis (0..2) with dt/h = lam, then (relax) the
// pressure relaxation; from_prim: in[] holds the primitive fields (as for
// launch_hyp_cons); to_prim: write the primitive fields and count bad cells
// into bad_row.  in and out must not overlap.
void launch_hyp_sweep(hipStream_t s, const DevGrid& g, const DevPhases& ph, int axis, double lam, int relax,
                      const double* const in[9], double* const out[9], int from_prim, int to_prim,
                      double* bad_row);
// max over cells and axes of (|u_d| + c) * ih[d] (ih[d] = 0 skips the axis) into rate_row.
void launch_hyp_rate(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* const prim[9],
                     const double ih[3], double* rate_row);

void launch_adj_cell(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* Tit,
                     const double* alpha2, const double* m1, const double* m2, const double* gLam,
                     const double* dg, const double* lam0, double* acc, double* mu, int first_pass,
                     const double* rCpsi, double* k0a, double* k0b, int init);

// Viscous heating by one velocity component (Sec. 3.2, phase internal
// energies): with the predicted velocity uh (uh64, or g64 + w32 in the FP32
// correction form) and the cell viscosity mu, phase k of cell a gains
//   tau sum_f 1/2 w_f alpha_k,f mu_f (uh_b - uh_a)^2
// (g.w carries the 4/3 factor of the component's own axis), which is the
// paper's flux form with face values uh_f = (uh_a+uh_b)/2 and alpha_k,f the
// arithmetic face mean; T_k += that / C_k, and in a cell without phase k the
// phase present takes both shares.  T1, T2 in place (T1 == NULL: no
// heating).  With E != NULL also the total-energy update of the viscous
// part, E += tau sum_f w_f mu_f uh_f (uh_b - uh_a).
void launch_visc_heat(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, int face, double tau,
                      const double* alpha2, const double* m1, const double* m2, const double* mu,
                      const double* uh64, const double* g64, const float* w32, double* T1, double* T2,
                      double* E);
// Total energy of the heat part: E += (T - Tn) / rC, rC = 1/C_eff of the
// pass whose final stage wrote T.
void launch_total_energy_heat(hipStream_t s, int64_t N, const double* T, const double* Tn, const double* rC,
                              double* E);

// One heat step of a 2D grid without sources and with equal p_inf in a
// single cooperative launch (tlim_step2d.hip): relaxation, then `passes`
// Picard passes, each with its P computed on the device from lambda_G.
constexpr int kStepMaxTiles = 4096;
struct Step2D {
    const double* alpha2;
    const double* T1;
    const double* T2;
    const double* m1;
    const double* m2;
    double* Tn;        // relaxed T (= g), all cells
    double* a2n;       // relaxed alpha2
    double* rC;        // 1/C_eff
    double* Tout[2];   // pass it writes T^(it+1) to Tout[it & 1]
    double* vx[2];     // exchange buffers between blocks of stages
    double* acc;       // accumulator rows (pass rows, kTgtFlag, kTgtP0..)
    unsigned* bar;     // kStepMaxTiles arrival words, zero before the launch
    const double* chat;  // b/lambda of P at chat + (P-1)^2, P = 1..pmax
    int pmax;
    int passes;
    unsigned spin_limit;  // polls a barrier wait may take before it counts a time-out
};
// Tiles the whole-step kernel uses on grid g (0 if it does not apply: fewer
// than 128 rows, or more tiles than can be resident at once).
int step2d_tiles(const DevGrid& g);
// Enqueue the step; false if the cooperative launch was refused (nothing ran).
bool launch_step2d(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                   const Step2D& st);

// Argument checks and packing shared by the context entry points and the
// context-free one (tlim_runtime.cpp): NULL when valid, else the reason.
const char* check_grid(const tlim_grid* g);
const char* check_phase(const tlim_phase* p);
DevPhases pack_phases(const tlim_phase ph[2]);
DevGrid pack_grid(const tlim_grid* g);
// Message of the last failing context-free call on the calling thread
// (returned by tlim_last_error(NULL)).
void set_free_error(const char* msg);

void launch_fill(hipStream_t s, double* p, double v, int64_t n);
void launch_copy(hipStream_t s, double* dst, const double* src, int64_t n);
void launch_widen(hipStream_t s, double* dst, const float* src, int64_t n);
void launch_narrow(hipStream_t s, float* dst, const double* src, int64_t n);

}  // namespace tlim
