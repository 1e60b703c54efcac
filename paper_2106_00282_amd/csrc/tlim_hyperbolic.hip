// Hyperbolic part of the six-equation model (Sec. 3.1: Godunov method with
// HLLC faces and dimensional splitting) and the pressure relaxation that
// follows it (Sec. 3.3), on gfx950.
//
// State: the conservative vector U of eq. vectorForm as nine double arrays,
// one per component, x fastest: alpha_1 rho_1, alpha_2 rho_2, rho u, rho v,
// rho w, alpha_1 rho_1 e_1, alpha_2 rho_2 e_2, rho E, alpha_2.
//
// A sweep along axis D runs one work-item per cell.  It loads its own cell
// and its two neighbours along D (27 doubles; the neighbours are the
// adjacent work-items' own cells and come from cache: along x within the
// wave, along y and z from the rows that the waves of the same block and the
// blocks before it load), solves the Riemann problems of its two faces,
// updates the cell, relaxes its pressure and writes nine doubles.  Every face
// is solved by both cells that share it: about twice the arithmetic of a
// face pass, for one pass over memory instead of two.  The last sweep of a
// step writes the library's primitive fields (alpha_2, m_k, T_k, velocity,
// rho E) instead of U and counts the cells that left the admissible range.
#include <hip/hip_runtime.h>
#include <math.h>

#include "tlim_internal.h"

namespace tlim {

namespace {

constexpr int NQ = 9;
constexpr int kHypThreads = 256;

// alpha_k p_k from the partial energy and mass of phase k (eq. eos_stiffened).
__device__ __forceinline__ double alpha_p(const DevPhases& ph, int k, double ak, double mk, double Ek) {
    return (ph.gamma[k] - 1.0) * (Ek - mk * ph.qf[k]) - ph.gamma[k] * ak * ph.pinf[k];
}

struct Mix {
    double rho, un, p, c;
};

// Mixture density, normal velocity, pressure sum_k alpha_k p_k and the speed
// of sound of the model, c^2 = Y_1 c_1^2 + Y_2 c_2^2 (Sec. 3.1), written as
// rho c^2 = sum_k gamma_k alpha_k (p_k + p_inf,k).
template <int D>
__device__ __forceinline__ Mix mixture(const DevPhases& ph, const double* q) {
    Mix s;
    const double a2 = q[8], a1 = 1.0 - a2;
    s.rho = q[0] + q[1];
    s.un = q[2 + D] / s.rho;
    const double ap1 = alpha_p(ph, 0, a1, q[0], q[5]);
    const double ap2 = alpha_p(ph, 1, a2, q[1], q[6]);
    s.p = ap1 + ap2;
    const double rc2 = ph.gamma[0] * (ap1 + a1 * ph.pinf[0]) + ph.gamma[1] * (ap2 + a2 * ph.pinf[1]);
    s.c = sqrt(rc2 / s.rho);
    return s;
}

// HLLC face between qL and qR along D (Davis speed estimates).  F is the
// flux u U + p D of eq. vectorForm at the face state, uf the face velocity
// u* of the non-conservative terms.  Star states scale every advected
// density by (S_K - u_K)/(S_K - S*) (phase masses, tangential momenta and
// phase internal energies, whose specific values cross the waves), keep
// alpha_2, set the normal momentum to rho* S* and give rho E the HLLC jump.
template <int D>
__device__ __forceinline__ void hllc(const DevPhases& ph, const double* qL, const double* qR, double* F,
                                     double& uf) {
    const Mix L = mixture<D>(ph, qL), R = mixture<D>(ph, qR);
    const double SL = fmin(L.un - L.c, R.un - R.c);
    const double SR = fmax(L.un + L.c, R.un + R.c);
    const double Ss = (R.p - L.p + L.rho * L.un * (SL - L.un) - R.rho * R.un * (SR - R.un)) /
                      (L.rho * (SL - L.un) - R.rho * (SR - R.un));
    double U[NQ], pf;
    if (SL >= 0.0) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) U[c] = qL[c];
        uf = L.un;
        pf = L.p;
    } else if (SR <= 0.0) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) U[c] = qR[c];
        uf = R.un;
        pf = R.p;
    } else {
        const bool kl = Ss >= 0.0;
        const double SK = kl ? SL : SR, uK = kl ? L.un : R.un, rK = kl ? L.rho : R.rho, pK = kl ? L.p : R.p;
        const double f = (SK - uK) / (SK - Ss);
#pragma unroll
        for (int c = 0; c < NQ; ++c) U[c] = (kl ? qL[c] : qR[c]) * f;
        U[2 + D] = rK * f * Ss;
        U[7] = f * ((kl ? qL[7] : qR[7]) + (Ss - uK) * (rK * Ss + pK / (SK - uK)));
        U[8] = kl ? qL[8] : qR[8];
        uf = Ss;
        pf = pK + rK * (SK - uK) * (Ss - uK);
    }
#pragma unroll
    for (int c = 0; c < NQ; ++c) F[c] = uf * U[c];
    F[2 + D] += pf;
    F[7] += pf * uf;
}

// Pressure relaxation of one state (Sec. 3.3).  Step 1: with the phase
// masses fixed and d(alpha_k rho_k e_k) = -p d alpha_k integrated at the
// relaxed pressure p, the SG EOS gives alpha_k(p) = k_k (A_k + p alpha_k^0) /
// (p + p_inf,k), k_k = (gamma_k - 1)/gamma_k, A_k = alpha_k rho_k (e_k - q_k);
// the saturation alpha_1(p) + alpha_2(p) = 1 is the quadratic
// (p + P1)(p + P2) = k_1 (A_1 + p a_1)(p + P2) + k_2 (A_2 + p a_2)(p + P1),
// whose larger root is the one above -min(P1, P2) (the other lies below).
// Step 2: the pressure of the SG mixture at these volume fractions from
// rho e = rho E - rho |u|^2 / 2.  Step 3: the phase energies at it.
__device__ __forceinline__ void relax_pressure(const DevPhases& ph, double* q) {
    const double a20 = q[8], a10 = 1.0 - a20;
    const double g1 = ph.gamma[0], g2 = ph.gamma[1], P1 = ph.pinf[0], P2 = ph.pinf[1];
    const double A1 = q[5] - q[0] * ph.qf[0], A2 = q[6] - q[1] * ph.qf[1];
    const double k1 = (g1 - 1.0) / g1, k2 = (g2 - 1.0) / g2;
    const double qa = 1.0 - k1 * a10 - k2 * a20;
    const double qb = P1 + P2 - k1 * (A1 + a10 * P2) - k2 * (A2 + a20 * P1);
    const double qc = P1 * P2 - k1 * A1 * P2 - k2 * A2 * P1;
    const double disc = fmax(qb * qb - 4.0 * qa * qc, 0.0);
    const double qq = -0.5 * (qb + copysign(sqrt(disc), qb));
    const double r1 = qq / qa;
    const double p1 = qq != 0.0 ? fmax(r1, qc / qq) : r1;
    const double a1 = k1 * (A1 + p1 * a10) / (p1 + P1);
    const double a2 = 1.0 - a1;
    const double rho = q[0] + q[1];
    const double ke = 0.5 * (q[2] * q[2] + q[3] * q[3] + q[4] * q[4]) / rho;
    const double rhoe = q[7] - ke;
    const double num = rhoe - q[0] * ph.qf[0] - q[1] * ph.qf[1] - a1 * g1 * P1 / (g1 - 1.0) - a2 * g2 * P2 / (g2 - 1.0);
    const double den = a1 / (g1 - 1.0) + a2 / (g2 - 1.0);
    const double p2 = num / den;
    q[5] = a1 * (p2 + g1 * P1) / (g1 - 1.0) + q[0] * ph.qf[0];
    q[6] = a2 * (p2 + g2 * P2) / (g2 - 1.0) + q[1] * ph.qf[1];
    q[8] = a2;
}

struct HypArgs {
    const double* in[NQ];  // U (or, for k_hyp_cons, the primitive fields)
    double* out[NQ];       // U, or the primitive fields when to_prim
    DevPhases ph;
    int nx, ny, nz;
    int64_t N, stride;     // cells; index step along the sweep axis
    int n, per;            // cells along the axis; periodic axis
    double lam;            // dt / h
    int relax, to_prim;
    double* bad;           // accumulator row of the count of inadmissible cells (to_prim)
};

// Primitive fields of the library in component order: m1, m2, u, v, w, T1,
// T2, rho E, alpha2 (out[] of the last sweep, in[] of k_hyp_cons).
template <int D>
__global__ void __launch_bounds__(kHypThreads) k_hyp_sweep(HypArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kHypThreads + threadIdx.x;
    double bad = 0.0;
    if (i < a.N) {
        const int64_t nxy = (int64_t)a.nx * a.ny;
        const int pos = D == 0 ? (int)(i % a.nx) : (D == 1 ? (int)((i / a.nx) % a.ny) : (int)(i / nxy));
        double qc[NQ], qm[NQ], qp[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qc[c] = a.in[c][i];
        // neighbours: the next cell along D, wrapped on a periodic axis, or the
        // mirror image of this cell behind a wall (normal momentum reversed)
        const bool hasm = pos > 0 || a.per, hasp = pos < a.n - 1 || a.per;
        const int64_t jm = pos > 0 ? i - a.stride : i + (int64_t)(a.n - 1) * a.stride;
        const int64_t jp = pos < a.n - 1 ? i + a.stride : i - (int64_t)(a.n - 1) * a.stride;
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            qm[c] = hasm ? a.in[c][jm] : qc[c];
            qp[c] = hasp ? a.in[c][jp] : qc[c];
        }
        if (!hasm) qm[2 + D] = -qc[2 + D];
        if (!hasp) qp[2 + D] = -qc[2 + D];
        double Fm[NQ], Fp[NQ], um, up;
        hllc<D>(a.ph, qm, qc, Fm, um);
        hllc<D>(a.ph, qc, qp, Fp, up);
        const double a2 = qc[8], a1 = 1.0 - a2;
        // non-conservative terms R(U_i) (u*_{i+1/2} - u*_{i-1/2})
        const double du = up - um;
        double R[NQ] = {0.0, 0.0, 0.0, 0.0, 0.0, alpha_p(a.ph, 0, a1, qc[0], qc[5]),
                        alpha_p(a.ph, 1, a2, qc[1], qc[6]), 0.0, -a2};
        double q[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q[c] = qc[c] - a.lam * (Fp[c] - Fm[c]) - a.lam * R[c] * du;
        if (a.relax) relax_pressure(a.ph, q);
        if (a.to_prim) {
            const double b2 = q[8], b1 = 1.0 - b2, rho = q[0] + q[1];
            const double T1 = (q[5] - q[0] * a.ph.qf[0] - b1 * a.ph.pinf[0]) / (q[0] * a.ph.cv[0]);
            const double T2 = (q[6] - q[1] * a.ph.qf[1] - b2 * a.ph.pinf[1]) / (q[1] * a.ph.cv[1]);
            a.out[0][i] = q[0];
            a.out[1][i] = q[1];
            a.out[2][i] = q[2] / rho;
            a.out[3][i] = q[3] / rho;
            a.out[4][i] = q[4] / rho;
            a.out[5][i] = T1;
            a.out[6][i] = T2;
            a.out[7][i] = q[7];
            a.out[8][i] = b2;
            if (!(b2 > 0.0 && b2 < 1.0) || !(T1 > 0.0) || !(T2 > 0.0) || isinf(T1) || isinf(T2)) bad = 1.0;
        } else {
#pragma unroll
            for (int c = 0; c < NQ; ++c) a.out[c][i] = q[c];
        }
    }
    if (a.to_prim) {
        // every wave: one atomic per wave that saw a bad cell
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
        if ((threadIdx.x & 63) == 0 && bad != 0.0) {
            const int sl = (int)(((int64_t)blockIdx.x * (kHypThreads / 64) + (threadIdx.x >> 6)) % kSlots);
            atomicAdd(a.bad + sl, bad);
        }
    }
}

// The library's state (alpha2, m_k, T_k, velocity, rho E) to U; in[2..4] and
// in[7] may be NULL (velocity 0; rho E from the state).  Pointwise, so out
// may alias in.
__global__ void __launch_bounds__(kHypThreads) k_hyp_cons(HypArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kHypThreads + threadIdx.x;
    if (i >= a.N) return;
    const double m1 = a.in[0][i], m2 = a.in[1][i];
    const double u = a.in[2] ? a.in[2][i] : 0.0, v = a.in[3] ? a.in[3][i] : 0.0, w = a.in[4] ? a.in[4][i] : 0.0;
    const double T1 = a.in[5][i], T2 = a.in[6][i], a2 = a.in[8][i], a1 = 1.0 - a2;
    const double rho = m1 + m2;
    const double E1 = m1 * (a.ph.cv[0] * T1 + a.ph.qf[0]) + a1 * a.ph.pinf[0];
    const double E2 = m2 * (a.ph.cv[1] * T2 + a.ph.qf[1]) + a2 * a.ph.pinf[1];
    const double Et = a.in[7] ? a.in[7][i] : E1 + E2 + 0.5 * rho * (u * u + v * v + w * w);
    a.out[0][i] = m1;
    a.out[1][i] = m2;
    a.out[2][i] = rho * u;
    a.out[3][i] = rho * v;
    a.out[4][i] = rho * w;
    a.out[5][i] = E1;
    a.out[6][i] = E2;
    a.out[7][i] = Et;
    a.out[8][i] = a2;
}

// Largest (|u_d| + c) / h_d over the cells and the axes with more than one
// cell, from the primitive fields (in[] as for k_hyp_cons), into a max row.
__global__ void __launch_bounds__(kHypThreads) k_hyp_rate(HypArgs a, double ihx, double ihy, double ihz,
                                                          double* rate) {
    const int64_t i = (int64_t)blockIdx.x * kHypThreads + threadIdx.x;
    double r = 0.0;
    if (i < a.N) {
        const double m1 = a.in[0][i], m2 = a.in[1][i];
        const double T1 = a.in[5][i], T2 = a.in[6][i], a2 = a.in[8][i], a1 = 1.0 - a2;
        const double rho = m1 + m2;
        const double E1 = m1 * (a.ph.cv[0] * T1 + a.ph.qf[0]) + a1 * a.ph.pinf[0];
        const double E2 = m2 * (a.ph.cv[1] * T2 + a.ph.qf[1]) + a2 * a.ph.pinf[1];
        const double ap1 = alpha_p(a.ph, 0, a1, m1, E1), ap2 = alpha_p(a.ph, 1, a2, m2, E2);
        const double rc2 = a.ph.gamma[0] * (ap1 + a1 * a.ph.pinf[0]) + a.ph.gamma[1] * (ap2 + a2 * a.ph.pinf[1]);
        const double c = sqrt(rc2 / rho);
        const double ih[3] = {ihx, ihy, ihz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double ud = a.in[2 + d] ? a.in[2 + d][i] : 0.0;
            if (ih[d] > 0.0) r = fmax(r, (fabs(ud) + c) * ih[d]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
    if ((threadIdx.x & 63) == 0) {
        const int sl = (int)(((int64_t)blockIdx.x * (kHypThreads / 64) + (threadIdx.x >> 6)) % kSlots);
        atomicMax((unsigned long long*)(rate + sl), (unsigned long long)__double_as_longlong(r + 0.0));
    }
}

unsigned hyp_blocks(int64_t N) { return (unsigned)((N + kHypThreads - 1) / kHypThreads); }

}  // namespace

void launch_hyp_cons(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* const prim[9],
                     double* const U[9]) {
    HypArgs a{};
    for (int c = 0; c < NQ; ++c) {
        a.in[c] = prim[c];
        a.out[c] = U[c];
    }
    a.ph = ph;
    a.N = g.N;
    hipLaunchKernelGGL(k_hyp_cons, dim3(hyp_blocks(g.N)), dim3(kHypThreads), 0, s, a);
}

void launch_hyp_sweep(hipStream_t s, const DevGrid& g, const DevPhases& ph, int axis, double lam, int relax,
                      const double* const in[9], double* const out[9], int to_prim, double* bad_row) {
    HypArgs a{};
    for (int c = 0; c < NQ; ++c) {
        a.in[c] = in[c];
        a.out[c] = out[c];
    }
    a.ph = ph;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.N = g.N;
    const int n[3] = {g.nx, g.ny, g.nz};
    a.n = n[axis];
    a.stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny);
    a.per = g.per[axis];
    a.lam = lam;
    a.relax = relax;
    a.to_prim = to_prim;
    a.bad = bad_row;
    const dim3 grid(hyp_blocks(g.N)), block(kHypThreads);
    if (axis == 0) hipLaunchKernelGGL(k_hyp_sweep<0>, grid, block, 0, s, a);
    else if (axis == 1) hipLaunchKernelGGL(k_hyp_sweep<1>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_hyp_sweep<2>, grid, block, 0, s, a);
}

void launch_hyp_rate(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* const prim[9],
                     const double ih[3], double* rate_row) {
    HypArgs a{};
    for (int c = 0; c < NQ; ++c) a.in[c] = prim[c];
    a.ph = ph;
    a.N = g.N;
    hipLaunchKernelGGL(k_hyp_rate, dim3(hyp_blocks(g.N)), dim3(kHypThreads), 0, s, a, ih[0], ih[1], ih[2],
                       rate_row);
}

}  // namespace tlim
