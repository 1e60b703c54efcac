// Hyperbolic part of the six-equation model (Sec. 3.1: Godunov method with
// HLLC faces and dimensional splitting) and the pressure relaxation that
// follows it (Sec. 3.3), on gfx950.
//
// State: the conservative vector U of eq. vectorForm as nine double arrays,
// one per component, x fastest: alpha_1 rho_1, alpha_2 rho_2, rho u, rho v,
// rho w, alpha_1 rho_1 e_1, alpha_2 rho_2 e_2, rho E, alpha_2.
//
// Every face's Riemann problem is solved once.  Along x a wave holds 64
// consecutive cells, one per lane; lane l solves the face between cells l-1
// (taken from the next lane down by DPP) and l, and the cell of lane l takes
// its right face from lane l+1 by DPP, so lanes 1..62 update their cells and
// a wave advances 62 cells per 64 loaded.  Along y and z a work-item owns a
// column segment of K cells at one x (a wave covers 64 consecutive x, so
// every load is a coalesced row) and marches along it, carrying the flux of
// the face behind it: K + 1 faces and K + 2 cell loads per K cells.  The
// update of a cell is then relaxed in pressure and written as U, or, in the
// last sweep of a step, as the library's primitive fields (alpha_2, m_k, T_k,
// velocity, rho E) with a count of the cells that left the admissible range.
#include <hip/hip_runtime.h>
#include <math.h>

#include "tlim_device.h"
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
    int from_prim;         // in[] holds the primitive fields: convert on load
    double* bad;           // accumulator row of the count of inadmissible cells (to_prim)
};

// U of cell i from the library's state (alpha2, m_k, T_k, velocity, rho E);
// in[2..4] and in[7] may be NULL (velocity 0; rho E from the state).
__device__ __forceinline__ void prim_to_cons(const HypArgs& a, int64_t i, double* q) {
    const double m1 = a.in[0][i], m2 = a.in[1][i];
    const double u = a.in[2] ? a.in[2][i] : 0.0, v = a.in[3] ? a.in[3][i] : 0.0, w = a.in[4] ? a.in[4][i] : 0.0;
    const double T1 = a.in[5][i], T2 = a.in[6][i], a2 = a.in[8][i], a1 = 1.0 - a2;
    const double rho = m1 + m2;
    const double E1 = m1 * (a.ph.cv[0] * T1 + a.ph.qf[0]) + a1 * a.ph.pinf[0];
    const double E2 = m2 * (a.ph.cv[1] * T2 + a.ph.qf[1]) + a2 * a.ph.pinf[1];
    q[0] = m1;
    q[1] = m2;
    q[2] = rho * u;
    q[3] = rho * v;
    q[4] = rho * w;
    q[5] = E1;
    q[6] = E2;
    q[7] = a.in[7] ? a.in[7][i] : E1 + E2 + 0.5 * rho * (u * u + v * v + w * w);
    q[8] = a2;
}

// Load U of cell i (converted from the state in the first sweep of a step).
__device__ __forceinline__ void load_cell(const HypArgs& a, int64_t i, double* q) {
    if (a.from_prim) {
        prim_to_cons(a, i, q);
        return;
    }
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[c] = a.in[c][i];
}

// Update of cell qc from its left and right face fluxes (eq. of the
// Godunov method in Sec. 3.1, with the non-conservative terms R(U_i)
// (u*_{i+1/2} - u*_{i-1/2}), R = (0, 0, 0, 0, 0, alpha_1 p_1, alpha_2 p_2,
// 0, -alpha_2)), the pressure relaxation, and the store: U, or the
// primitive fields with the admissibility check (returns 1 for a bad cell).
__device__ __forceinline__ double finish_cell(const HypArgs& a, int64_t i, const double* qc, const double* Fm,
                                              const double* Fp, double um, double up) {
    const double a2 = qc[8], a1 = 1.0 - a2;
    const double du = up - um;
    const double R[NQ] = {0.0, 0.0, 0.0, 0.0, 0.0, alpha_p(a.ph, 0, a1, qc[0], qc[5]),
                          alpha_p(a.ph, 1, a2, qc[1], qc[6]), 0.0, -a2};
    double q[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[c] = qc[c] - a.lam * (Fp[c] - Fm[c]) - a.lam * R[c] * du;
    if (a.relax) relax_pressure(a.ph, q);
    if (!a.to_prim) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) a.out[c][i] = q[c];
        return 0.0;
    }
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
    return (!(b2 > 0.0 && b2 < 1.0) || !(T1 > 0.0) || !(T2 > 0.0) || isinf(T1) || isinf(T2)) ? 1.0 : 0.0;
}

// One wave-level count of bad cells into a slot of the row.
__device__ __forceinline__ void count_bad(const HypArgs& a, double bad) {
    if (!a.to_prim) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad != 0.0) {
        const int sl = (int)(((int64_t)blockIdx.x * (kHypThreads / 64) + (threadIdx.x >> 6)) % kSlots);
        atomicAdd(a.bad + sl, bad);
    }
}

constexpr int kXOut = 62;  // cells a wave updates along x (lanes 1..62)

// Sweep along x.  Wave w of row r loads cells x = 62 t - 1 + lane of tile t
// (wrapped on a periodic axis; outside a wall the mirror image of the end
// cell, normal momentum reversed), every lane active.
__global__ void __launch_bounds__(kHypThreads) k_hyp_sweep_x(HypArgs a, int tiles_x, int64_t waves) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kHypThreads / 64) + (threadIdx.x >> 6);
    double bad = 0.0;
    if (wid < waves) {  // wave-uniform
        const int t = (int)(wid % tiles_x);
        const int64_t rowi = wid / tiles_x;
        const int nx = a.nx;
        const int xg = kXOut * t - 1 + lane;
        int xc = xg;
        bool mirror = false;
        if (a.per) {
            xc = xg % nx;
            if (xc < 0) xc += nx;
        } else if (xg < 0 || xg >= nx) {
            xc = xg < 0 ? 0 : nx - 1;
            mirror = true;
        }
        const int64_t base = rowi * nx;
        double qc[NQ];
        load_cell(a, base + xc, qc);
        if (mirror) qc[2] = -qc[2];
        // face between the cell of lane-1 and this lane's cell
        double qL[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qL[c] = tb::from_left(qc[c]);
        double F[NQ], uf;
        hllc<0>(a.ph, qL, qc, F, uf);
        double Fr[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) Fr[c] = tb::from_right(F[c]);
        const double ur = tb::from_right(uf);
        if (lane >= 1 && lane <= kXOut && xg < nx) bad = finish_cell(a, base + xg, qc, F, Fr, uf, ur);
    }
    count_bad(a, bad);
}

// Sweep along y (D = 1) or z (D = 2): a work-item marches along a column
// segment of K cells.
template <int D>
__global__ void __launch_bounds__(kHypThreads) k_hyp_sweep_col(HypArgs a, int K, int segs, int64_t items) {
    const int64_t it = (int64_t)blockIdx.x * kHypThreads + threadIdx.x;
    double bad = 0.0;
    if (it < items) {
        const int nx = a.nx;
        const int x = (int)(it % nx);
        const int64_t r = it / nx;
        const int seg = (int)(r % segs);
        const int64_t other = r / segs;  // z (for D = 1) or y (for D = 2)
        const int64_t s = a.stride;
        const int64_t col0 = D == 1 ? other * (int64_t)nx * a.ny + x : other * (int64_t)nx + x;
        const int n = a.n;
        const int j0 = seg * K;
        const int j1 = j0 + K < n ? j0 + K : n;
        // neighbour j of the column: wrapped, or the mirror of the end cell
        auto load_nb = [&](int j, double* q) {
            bool mirror = false;
            int jc = j;
            if (j < 0 || j >= n) {
                if (a.per) jc = j < 0 ? j + n : j - n;
                else {
                    jc = j < 0 ? 0 : n - 1;
                    mirror = true;
                }
            }
            load_cell(a, col0 + (int64_t)jc * s, q);
            if (mirror) q[2 + D] = -q[2 + D];
        };
        double qm[NQ], qc[NQ], qp[NQ], Fm[NQ], Fp[NQ], um, up;
        load_nb(j0 - 1, qm);
        load_cell(a, col0 + (int64_t)j0 * s, qc);
        hllc<D>(a.ph, qm, qc, Fm, um);
        for (int j = j0; j < j1; ++j) {
            load_nb(j + 1, qp);
            hllc<D>(a.ph, qc, qp, Fp, up);
            bad += finish_cell(a, col0 + (int64_t)j * s, qc, Fm, Fp, um, up);
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                qc[c] = qp[c];
                Fm[c] = Fp[c];
            }
            um = up;
        }
    }
    count_bad(a, bad);
}

// The library's state to U (pointwise, so out may alias in).
__global__ void __launch_bounds__(kHypThreads) k_hyp_cons(HypArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kHypThreads + threadIdx.x;
    if (i >= a.N) return;
    double q[NQ];
    prim_to_cons(a, i, q);
#pragma unroll
    for (int c = 0; c < NQ; ++c) a.out[c][i] = q[c];
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
                      const double* const in[9], double* const out[9], int from_prim, int to_prim,
                      double* bad_row) {
    HypArgs a{};
    a.from_prim = from_prim;
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
    const dim3 block(kHypThreads);
    if (axis == 0) {
        const int tiles_x = (g.nx + kXOut - 1) / kXOut;
        const int64_t waves = (int64_t)tiles_x * g.ny * g.nz;
        const int64_t blocks = (waves + kHypThreads / 64 - 1) / (kHypThreads / 64);
        hipLaunchKernelGGL(k_hyp_sweep_x, dim3((unsigned)blocks), block, 0, s, a, tiles_x, waves);
        return;
    }
    // column segments of K cells, as long as about 2^17 work-items (two
    // waves per SIMD) remain, at most 16: fewer halo loads per cell against
    // fewer waves in flight (at 1024^2, K = 8 takes 4% less time than
    // K = 4 and 8% less than K = 2)
    const int64_t cols = g.N / a.n;
    int64_t K = g.N / ((int64_t)1 << 17);
    K = K < 1 ? 1 : (K > 16 ? 16 : K);
    if (K > a.n) K = a.n;
    const int segs = (int)((a.n + K - 1) / K);
    const int64_t items = cols * segs;
    const dim3 grid(hyp_blocks(items));
    if (axis == 1) hipLaunchKernelGGL(k_hyp_sweep_col<1>, grid, block, 0, s, a, (int)K, segs, items);
    else hipLaunchKernelGGL(k_hyp_sweep_col<2>, grid, block, 0, s, a, (int)K, segs, items);
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
