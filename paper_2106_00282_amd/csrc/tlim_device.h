// Device helpers shared by the kernel files: the material laws (all
// kernels) and the wave-level tools of the 2D kernels that keep one column
// per lane (blocked stages in tlim_sweep.hip, reverse stages in
// tlim_adjoint.hip, 2D coefficients in tlim_coeffs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "tlim_internal.h"

namespace tlim {
namespace phys {

// Out-of-line pieces of the cell laws: a general power, the logarithm, the
// relaxation of an interface cell and the interface term of 1/C.  The 2D
// kernels evaluate the laws for 8 rows per lane in one-shot prologues and
// epilogues; inlined, every row carries its own copy of this code, the
// kernels grow past the instruction cache and that straight-line code runs
// at the pace of instruction fetch.  Called, one copy serves every row.
// Arguments are scalars: a reference to a kernel argument would copy the
// whole argument block to scratch memory.
static __device__ __attribute__((noinline)) double pow_ool(double x, double n) { return pow(x, n); }
static __device__ __attribute__((noinline)) double log_ool(double x) { return log(x); }

// (T/T0)^n with the exponents the conductivity laws use written out, so the
// common integer and half-integer cases are exact products.
static __device__ __forceinline__ double powlaw(double x, double n) {
    if (n == 0.0) return 1.0;
    if (n == 1.0) return x;
    if (n == 2.0) return x * x;
    if (n == 3.0) return x * x * x;
    if (n == 2.5) return x * x * sqrt(x);
    return pow_ool(x, n);
}

static __device__ __forceinline__ bool is_mixed(double a2, double eps) { return a2 > eps && a2 < 1.0 - eps; }

// W = Gamma_1 C_1/alpha_1^2 + Gamma_2 C_2/alpha_2^2 (interface cells).
static __device__ __forceinline__ double pressure_stiffness(const DevPhases& ph, double a2, double C1, double C2) {
    double a1 = 1.0 - a2;
    return (ph.gamma[0] - 1.0) * C1 / (a1 * a1) + (ph.gamma[1] - 1.0) * C2 / (a2 * a2);
}

// Coulomb logarithm of the Spitzer-Harm law (Sec. 4.4) from ln T and
// ln rho: ln(l_D / max(l_LD, l_dB)), floored at 1, with ln l_D =
// ln sh_D + (ln T - ln rho)/2, ln l_LD = ln sh_LD - ln T and
// ln l_dB = ln sh_dB - ln T / 2.  slope = d ln(ln Lambda)/d ln T times
// ln Lambda: 3/2 with the Landau length, 1 with the de Broglie length, 0 on
// the floor.
static __device__ __forceinline__ double coulomb_log(const DevPhases& ph, int k, double lt, double lr,
                                                     double& slope) {
    const double lld = ph.ln_shLD[k] - lt, ldb = ph.ln_shdB[k] - 0.5 * lt;
    const double L = ph.ln_shD[k] + 0.5 * (lt - lr) - fmax(lld, ldb);
    slope = L > 1.0 ? (lld >= ldb ? 1.5 : 1.0) : 0.0;
    return L > 1.0 ? L : 1.0;
}

// ln T and ln rho for the Spitzer-Harm law (unused otherwise).
struct LawLogs {
    double lt, lr;
};
static __device__ __forceinline__ LawLogs law_logs(const DevPhases& ph, double t, double rho) {
    LawLogs g{0.0, 0.0};
    if (ph.spitzer) {
        g.lt = log_ool(t);
        g.lr = log_ool(rho);
    }
    return g;
}

// Mixture density rho = m1 + m2 of cell i, read only when a phase uses the
// Spitzer-Harm law (the power law does not depend on it).
template <typename I>
static __device__ __forceinline__ double mix_density(const DevPhases& ph, const double* m1, const double* m2, I i) {
    return ph.spitzer ? m1[i] + m2[i] : 1.0;
}

// lambda_k / k0_k of phase k: (T/T0)^n, over ln Lambda_ei under the
// Spitzer-Harm law.
static __device__ __forceinline__ double phase_law(const DevPhases& ph, int k, double t, const LawLogs& g) {
    double x = powlaw(t * ph.invT0[k], ph.npow[k]);
    if (ph.sh_law[k]) {
        double slope;
        x /= coulomb_log(ph, k, g.lt, g.lr, slope);
    }
    return x;
}

// d lambda_k / dT of phase k at fixed rho.
static __device__ __forceinline__ double phase_law_dT(const DevPhases& ph, int k, double t, const LawLogs& g) {
    const double x = t * ph.invT0[k];
    double d = ph.npow[k] != 0.0 ? ph.k0[k] * ph.npow[k] * powlaw(x, ph.npow[k] - 1.0) * ph.invT0[k] : 0.0;
    if (ph.sh_law[k]) {
        double slope;
        const double L = coulomb_log(ph, k, g.lt, g.lr, slope);
        d = (d - ph.k0[k] * powlaw(x, ph.npow[k]) * slope / (t * L)) / L;
    }
    return d;
}

// Derivatives of the cell conductivity at (rho, T) for the adjoint:
// dk[k] = d Lambda / d k0_k = alpha_k lambda_k / k0_k and dT = d Lambda / dT.
static __device__ __forceinline__ void cell_conductivity_grad(const DevPhases& ph, double t, double a2, double rho,
                                                              double dk[2], double& dT) {
    const LawLogs g = law_logs(ph, t, rho);
    const double a1 = 1.0 - a2;
    dk[0] = a1 * phase_law(ph, 0, t, g);
    dk[1] = a2 * phase_law(ph, 1, t, g);
    dT = a1 * phase_law_dT(ph, 0, t, g) + a2 * phase_law_dT(ph, 1, t, g);
}

// Cell conductivity Lambda = sum_k alpha_k lambda_k(rho, T) (eq. qk_dis);
// rho (the mixture density) matters only under the Spitzer-Harm law.
static __device__ __forceinline__ double cell_conductivity(const DevPhases& ph, double t, double a2, double rho) {
    const LawLogs g = law_logs(ph, t, rho);
    return (1.0 - a2) * (ph.k0[0] * phase_law(ph, 0, t, g)) + a2 * (ph.k0[1] * phase_law(ph, 1, t, g));
}

// The same when neither phase uses the Spitzer-Harm law (bitwise equal to
// cell_conductivity there).
static __device__ __forceinline__ double cell_conductivity_pow(const DevPhases& ph, double t, double a2) {
    return (1.0 - a2) * (ph.k0[0] * powlaw(t * ph.invT0[0], ph.npow[0])) +
           a2 * (ph.k0[1] * powlaw(t * ph.invT0[1], ph.npow[1]));
}

// Lambda of cell i in kernels compiled per law family: kSH when a phase
// follows the Spitzer-Harm law (rho = m1 + m2 read), else the power law
// only, so that the power-law kernels carry no logarithms.
template <bool kSH, typename I>
static __device__ __forceinline__ double cell_lambda(const DevPhases& ph, double t, double a2, const double* m1,
                                                     const double* m2, I i) {
    if constexpr (kSH) return cell_conductivity(ph, t, a2, m1[i] + m2[i]);
    else return cell_conductivity_pow(ph, t, a2);
}

// B1^2 / (T^2 W) of an interface cell, with W of pressure_stiffness.
static __device__ __attribute__((noinline)) double interface_capacity(double B1, double gam0, double gam1, double t,
                                                                      double a2, double C1, double C2) {
    const double a1 = 1.0 - a2;
    const double W = (gam0 - 1.0) * C1 / (a1 * a1) + (gam1 - 1.0) * C2 / (a2 * a2);
    return B1 * B1 / (t * t * W);
}

// 1 / C_eff (Sec. 3.4.2 under T_1 = T_2 and p_1 = p_2).
static __device__ __forceinline__ double inv_heat_capacity(const DevPhases& ph, double eps, double t, double a2,
                                                           double m1, double m2) {
    double B1 = ph.pinf[0] - ph.pinf[1];
    double C1 = m1 * ph.cv[0], C2 = m2 * ph.cv[1];
    double C = C1 + C2;
    if (B1 != 0.0 && is_mixed(a2, eps)) C += interface_capacity(B1, ph.gamma[0], ph.gamma[1], t, a2, C1, C2);
    return 1.0 / C;
}

// End state of the relaxation system in an interface cell (Sec. 3.4.1):
// phase energies summed conserve E = C1 T1 + C2 T2 + alpha_k p_inf,k, and
// p_1 = p_2 at T_1 = T_2 = T'.  With B = p_inf,2 - p_inf,1,
// T'(a) = (C1 T1 + C2 T2 + (alpha2^0 - a) B)/(C1 + C2) and
// (p_1 - p_2) a (1-a) = A2 a^2 + A1 a + A0 is quadratic in a = alpha2'.
// The root with 0 < a < 1 and T'(a) > 0 is taken (eq. Taverage when B = 0).
// Interface cell (eps < alpha2^0 < 1 - eps) of relax_cell.
struct Relaxed {
    double T, a2;
};
static __device__ __attribute__((noinline)) Relaxed relax_interface(double pinf0, double pinf1, double gam0,
                                                                    double gam1, double cv0, double cv1,
                                                                    double a20, double T1, double T2, double m1,
                                                                    double m2) {
    const double B = pinf1 - pinf0;
    const double G1 = gam0 - 1.0, G2 = gam1 - 1.0;
    double C1 = m1 * cv0, C2 = m2 * cv1;
    double S = C1 + C2;
    double E = C1 * T1 + C2 * T2;
    double t0 = (E + a20 * B) / S, t1 = -B / S;   // T'(a) = t0 + t1 a
    double l0 = -G2 * C2, l1 = G1 * C1 + G2 * C2;  // L(a) = l0 + l1 a
    double A2 = t1 * l1 - B, A1 = t0 * l1 + t1 * l0 + B, A0 = t0 * l0;
    double root;
    if (A2 == 0.0) {
        root = -A0 / A1;
    } else {
        double disc = fmax(A1 * A1 - 4.0 * A2 * A0, 0.0);
        double qq = -0.5 * (A1 + copysign(sqrt(disc), A1));
        double r1 = qq / A2, r2 = A0 / qq;
        bool ok1 = r1 > 0.0 && r1 < 1.0 && t0 + t1 * r1 > 0.0;
        bool ok2 = r2 > 0.0 && r2 < 1.0 && t0 + t1 * r2 > 0.0;
        root = ok1 ? r1 : r2;
        if (ok1 && ok2) root = fabs(r1 - a20) < fabs(r2 - a20) ? r1 : r2;
        if (!ok1 && !ok2) {
            // rounding pushed the admissible root out: bisect the sign change
            // of the quadratic on (lo, hi) = {0 < a < 1, T'(a) > 0}
            double lo = 0.0, hi = 1.0;
            if (t1 < 0.0) hi = fmin(hi, -t0 / t1);
            if (t1 > 0.0) lo = fmax(lo, -t0 / t1);
            for (int it = 0; it < 120; ++it) {
                double mid = 0.5 * (lo + hi);
                if ((A2 * mid + A1) * mid + A0 < 0.0) lo = mid;
                else hi = mid;
            }
            root = 0.5 * (lo + hi);
        }
        // two Newton steps on the quadratic polish the root
        for (int it = 0; it < 2; ++it) {
            double f = (A2 * root + A1) * root + A0, df = 2.0 * A2 * root + A1;
            if (df != 0.0) root -= f / df;
        }
    }
    return Relaxed{t0 + t1 * root, root};
}

static __device__ __forceinline__ void relax_cell(const DevPhases& ph, double eps, double a20, double T1,
                                                  double T2, double m1, double m2, double& T, double& a2) {
    if (a20 <= eps || a20 >= 1.0 - eps) {
        // pure cell: the absent phase takes the present phase's temperature
        T = a20 <= eps ? T1 : T2;
        a2 = a20;
        return;
    }
    const Relaxed r = relax_interface(ph.pinf[0], ph.pinf[1], ph.gamma[0], ph.gamma[1], ph.cv[0], ph.cv[1], a20,
                                      T1, T2, m1, m2);
    T = r.T;
    a2 = r.a2;
}

}  // namespace phys

namespace tb {

// Extended tile: 64 lanes (x) by WAVES waves of ROWS rows (y) per workgroup;
// up to KMAX stages per launch.
constexpr int KMAX = 8;
constexpr int WAVES = 8;
constexpr int ROWS = 8;
constexpr int EXT_Y = WAVES * ROWS;

// Lane i receives lane i-1 (wave_shr:1) or lane i+1 (wave_shl:1); with
// bound_ctrl the lanes at the ends receive 0 (they are halo lanes).
static __device__ __forceinline__ int dpp_from_left(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true); }
static __device__ __forceinline__ int dpp_from_right(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true); }

static __device__ __forceinline__ double from_left(double x) {
    return __hiloint2double(dpp_from_left(__double2hiint(x)), dpp_from_left(__double2loint(x)));
}
static __device__ __forceinline__ double from_right(double x) {
    return __hiloint2double(dpp_from_right(__double2hiint(x)), dpp_from_right(__double2loint(x)));
}
static __device__ __forceinline__ float from_left(float x) { return __int_as_float(dpp_from_left(__float_as_int(x))); }
static __device__ __forceinline__ float from_right(float x) { return __int_as_float(dpp_from_right(__float_as_int(x))); }

template <typename R>
static __device__ __forceinline__ R fmean(R a, R b, int face) {
    if (face == 1) {
        R s = a + b;
        return s > R(0) ? R(2) * (a * b) / s : R(0);
    }
    return R(0.5) * (a + b);
}

// Index of an unwrapped coordinate: wrap on a periodic axis, clamp on an
// adiabatic one (clamped copies only feed halo cells, whose wall faces
// carry kappa = 0).
static __device__ __forceinline__ int fold(int c, int n, int per) {
    if (per) {
        int m = c % n;
        return m < 0 ? m + n : m;
    }
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Folded index of row yg0 + r, given yi0 = fold(yg0): the grids blocked
// by rows have at least ROWS rows, so a periodic row wraps at most once.
static __device__ __forceinline__ int row_index(int yi0, int yg0, int r, int ny, int per) {
    if (per) {
        const int y = yi0 + r;
        return y >= ny ? y - ny : y;
    }
    const int y = yg0 + r;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// This workgroup's place in an order in which each of the 8 XCDs (each with
// an L2 of its own, and given workgroups in turn) runs a contiguous run of
// places: XCD x runs floor(n/8) of them, one more for x < n mod 8.  Tiles
// taken in this order put most neighbours, whose halos overlap, on one L2.
static __device__ __forceinline__ int xcd_block() {
    const int nb = (int)gridDim.x, x = (int)blockIdx.x & 7;
    return x * (nb >> 3) + min(x, nb & 7) + ((int)blockIdx.x >> 3);
}

// Lane l's value of a double (l wave-uniform), without memory access.
static __device__ __forceinline__ double lane_value(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

}  // namespace tb
}  // namespace tlim
