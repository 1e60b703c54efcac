/*
 * FP64 CPU oracle of the parabolic sub-step (arXiv 2106.00282, Sec. 3.2 and
 * Sec. 3.4, Algorithm 1), and of the mechanical stage before it (hyperbolic
 * part and pressure relaxation, Sec. 3.1 and Sec. 3.3).  TEST
 * INFRASTRUCTURE ONLY: the product path never links or calls it.  See
 * tlim_oracle.h for the scope, the pins and what is left unpinned.
 *
 * Readings of the paper taken here (each one is also listed with its reason
 * in the design notes of the repository):
 *  - Chebyshev roots: beta_1 = cos(pi/2P) is the largest root, so that
 *    a_1 = 0 < a_2 < ... < a_P (Sec. 3.2, parameters of eq. LIM).
 *  - Stage order: the same multiset of parameters as the paper, in the
 *    order (a_P, a_2, a_{P-1}, a_3, ...) twice with a_1 = 0 last.  Every
 *    stage has the fixed point (I + tau A)^-1 g and the stage maps commute,
 *    so in exact arithmetic every order gives the same result; in floating
 *    point the printed order (a_P..a_2, a_P..a_1) and ascending pairs let
 *    round-off grow by many orders of magnitude at tau*lambda = 400 on a
 *    grid, the interleaved order does not.  Both others stay as options.
 *  - v^(0) = v^n; the operator L_h of eq. LIM is -A with A = C^-1 D >= 0,
 *    the final stage is v^n - tau A v_hat + tau f in flux form (eq. LIM_last).
 *  - lambda_max is the Gershgorin bound of A, taken per Picard pass.
 *  - Face conductivity: arithmetic mean of the cell values
 *    Lambda = sum_k alpha_k lambda_k(T) (eq. qk_dis leaves it open).
 *  - Heat step: with T_1 = T_2 = T and p_1 = p_2 held, the phase energy
 *    equations reduce to C_eff dT/dt = sum_k (q_k + I_k), with
 *    C_eff = C_1 + C_2 + B_1^2/(T^2 W), W = G1 C1/a1^2 + G2 C2/a2^2, and
 *    d alpha_2/dT = -B_1/(T^2 W) (B_1 = p_inf,1 - p_inf,2).  For equal p_inf
 *    this is the mixture heat equation with alpha_2 frozen.
 *  - Temperature relaxation: the exact end state of the relaxation system
 *    (phase energies summed, p_1 = p_2, T_1 = T_2); for equal p_inf it is
 *    eq. Taverage.  The root with T' <= 0 is rejected.
 *  - Picard: every pass restarts the LIM from T^n with coefficients lagged
 *    at T^(it); err = max|T^(it+1) - T^(it)| / max|T^(it+1)|.
 *  - Spitzer-Harm law (Sec. 4.4): the Coulomb logarithm from the Debye,
 *    Landau and de Broglie lengths with caller-given constants, floored at
 *    1; rho is the cell's mixture density.
 *  - Hyperbolic part: Davis wave speeds, the model's sound speed, star
 *    states that scale every advected density by (S_K - u_K)/(S_K - S*);
 *    each directional sweep is followed by the pressure relaxation, whose
 *    step 1 integrates at the relaxed pressure; walls reflect.
 */
#include "tlim_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

static int64_t ncells(const orc_grid* g) { return g->n[0] * g->n[1] * g->n[2]; }

static double cell_volume(const orc_grid* g) { return g->h[0] * g->h[1] * g->h[2]; }

static double* dalloc(int64_t n) {
    double* p = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!p) abort();
    return p;
}

/* The faces of one cell: neighbour index and weight s_axis / h_axis^2.
 * A face exists towards the next cell along an axis, wrapping round on a
 * periodic axis; an adiabatic end and an axis of a single cell have none.
 * On a periodic axis of two cells both faces lead to the same neighbour. */
typedef struct {
    int count;
    int64_t nb[6];
    double w[6];
} cell_faces;

static void faces_of(const orc_grid* g, const double axis_scale[3], int64_t i, int64_t j, int64_t k,
                     cell_faces* f) {
    int64_t c[3] = {i, j, k};
    int64_t stride[3] = {1, g->n[0], g->n[0] * g->n[1]};
    int64_t a = i + g->n[0] * (j + g->n[1] * k);
    f->count = 0;
    for (int axis = 0; axis < 3; ++axis) {
        int64_t n = g->n[axis];
        if (n <= 1) continue;
        double w = axis_scale[axis] / (g->h[axis] * g->h[axis]);
        for (int dir = -1; dir <= 1; dir += 2) {
            int64_t cn = c[axis] + dir;
            if (cn < 0 || cn >= n) {
                if (g->bc[axis] != ORC_PERIODIC) continue;
                cn = (cn + n) % n;
            }
            f->nb[f->count] = a + (cn - c[axis]) * stride[axis];
            f->w[f->count] = w;
            f->count++;
        }
    }
}

static double face_value(double La, double Lb, int32_t face_mean) {
    if (face_mean == ORC_FACE_HARMONIC) {
        double s = La + Lb;
        return s > 0.0 ? 2.0 * (La * Lb) / s : 0.0;
    }
    return 0.5 * (La + Lb);
}

/* d Lambda_f / d Lambda_a for the face mean (the other side by symmetry). */
static double face_partial(double La, double Lb, int32_t face_mean) {
    if (face_mean == ORC_FACE_HARMONIC) {
        double s = La + Lb;
        return s > 0.0 ? 2.0 * Lb * Lb / (s * s) : 0.0;
    }
    return 0.5;
}

/* Coulomb logarithm of the Spitzer-Harm law (Sec. 4.4): ln(l_D / l_LD) when
 * the Landau length is at least the de Broglie length, else ln(l_D / l_dB),
 * and never below 1.  *landau says which length was taken, *floored whether
 * the floor applied. */
static double coulomb_log(const orc_phase* p, double T, double rho, int* landau, int* floored) {
    double lD = p->sh_D * sqrt(T / rho);
    double lLD = p->sh_LD / T;
    double ldB = p->sh_dB / sqrt(T);
    int lan = lLD >= ldB;
    double L = lan ? log(lD / lLD) : log(lD / ldB);
    if (landau) *landau = lan;
    if (floored) *floored = !(L > 1.0);
    return L > 1.0 ? L : 1.0;
}

/* lambda_k(rho, T) / k0: (T/T0)^n, divided by the Coulomb logarithm under the
 * Spitzer-Harm law. */
static double conductivity_per_k0(const orc_phase* p, double T, double rho) {
    double x = pow(T / p->T0, p->npow);
    if (p->law == ORC_LAW_SPITZER) x /= coulomb_log(p, T, rho, NULL, NULL);
    return x;
}

static double conductivity(const orc_phase* p, double T, double rho) {
    return p->k0 * conductivity_per_k0(p, T, rho);
}

/* d lambda_k / dT at fixed rho.  Under the Spitzer-Harm law, away from the
 * floor, d ln(ln Lambda)/d ln T = (1/2 + 1)/ln Lambda with the Landau length
 * (l_D grows as T^(1/2), l_LD falls as 1/T) and (1/2 + 1/2)/ln Lambda with
 * the de Broglie length (l_dB falls as T^(-1/2)). */
static double conductivity_dT(const orc_phase* p, double T, double rho) {
    double lam = p->k0 * pow(T / p->T0, p->npow);
    double dlog = p->npow / T; /* d ln lambda / dT of the power law */
    if (p->law == ORC_LAW_SPITZER) {
        int landau, floored;
        double L = coulomb_log(p, T, rho, &landau, &floored);
        lam /= L;
        if (!floored) dlog -= (landau ? 1.5 : 1.0) / (T * L);
    }
    return lam * dlog;
}

static double mixture_density(const double* m1, const double* m2, int64_t i) {
    return m1 && m2 ? m1[i] + m2[i] : 1.0;
}

/* ------------------------------------------------------------------------ */
/* Chebyshev parameters (Sec. 3.2, eq. LIM and the definition of a_m).       */

int32_t orc_lim_P(double tau, double lambda_max) {
    return (int32_t)ceil(PI / 4.0 * sqrt(tau * lambda_max + 1.0));
}

/* Large-small interleave of an increasing list x[0] < ... < x[n-1]:
 * x[n-1], x[0], x[n-2], x[1], ... */
static void interleave(const double* x, int32_t n, double* out) {
    int32_t lo = 0, hi = n - 1, k = 0, take_hi = 1;
    while (lo <= hi) {
        out[k++] = take_hi ? x[hi--] : x[lo++];
        take_hi = !take_hi;
    }
}

void orc_lim_params(int32_t P, double lambda_max, int32_t order, double* b) {
    /* beta_j = cos((2j-1) pi / (2P)), j = 1..P, beta_1 the largest root, and
     * a_j = lambda_max (beta_1 - beta_j) / (1 + beta_1), so a_1 = 0 < a_2 < ... < a_P. */
    double* a = dalloc(P + 1);
    double beta1 = cos(PI / (2.0 * P));
    for (int32_t j = 1; j <= P; ++j) {
        double betaj = cos((2.0 * j - 1.0) * PI / (2.0 * P));
        a[j] = lambda_max / (1.0 + beta1) * (beta1 - betaj);
    }
    a[1] = 0.0;
    int32_t k = 0;
    if (order == ORC_ORDER_PAPER) {
        /* (a_P, a_{P-1}, ..., a_2, a_P, a_{P-1}, ..., a_1) as printed */
        for (int32_t j = P; j >= 2; --j) b[k++] = a[j];
        for (int32_t j = P; j >= 1; --j) b[k++] = a[j];
    } else if (order == ORC_ORDER_ASCENDING) {
        /* (a_2, a_2, a_3, a_3, ..., a_P, a_P, a_1) */
        for (int32_t j = 2; j <= P; ++j) {
            b[k++] = a[j];
            b[k++] = a[j];
        }
        b[k++] = a[1];
    } else {
        /* (a_P, a_2, a_{P-1}, a_3, ...) twice, then a_1: the same multiset,
         * ordered so that no partial product of stage factors grows large. */
        if (P > 1) {
            interleave(a + 2, P - 1, b);
            interleave(a + 2, P - 1, b + (P - 1));
        }
        b[2 * P - 2] = a[1];
    }
    free(a);
}

void orc_cycle_params(int32_t s, double lambda_max, double* b) {
    /* Richardson steps 1/(1 + tau b_j) with 1 + tau b_j at the Chebyshev
     * nodes of [1, 1 + tau lambda_max]: b_j = lambda/2 (1 + cos((2j-1) pi/(2s))),
     * applied in increasing order (j = s, ..., 1), so that each cycle ends with
     * the stages that damp the high modes most and the residual reaches its
     * rounding floor. */
    for (int32_t k = 0; k < s; ++k) {
        int32_t j = s - k;
        b[k] = 0.5 * lambda_max * (1.0 + cos((2.0 * j - 1.0) * PI / (2.0 * s)));
    }
}

/* ------------------------------------------------------------------------ */
/* Coefficients (Sec. 3.4.2).                                                 */

void orc_cell_conductivity(const orc_grid* g, const orc_phase ph[2], const double* alpha2,
                           const double* m1, const double* m2, const double* T, double* Lam) {
    int64_t N = ncells(g);
    for (int64_t i = 0; i < N; ++i) {
        double a2 = alpha2[i], a1 = 1.0 - a2, rho = mixture_density(m1, m2, i);
        Lam[i] = a1 * conductivity(&ph[0], T[i], rho) + a2 * conductivity(&ph[1], T[i], rho);
    }
}

static int is_mixed(double a2, double eps) { return a2 > eps && a2 < 1.0 - eps; }

/* W = Gamma_1 C_1 / alpha_1^2 + Gamma_2 C_2 / alpha_2^2 (mixed cells). */
static double pressure_stiffness(const orc_phase ph[2], double a2, double C1, double C2) {
    double a1 = 1.0 - a2;
    return (ph[0].gamma - 1.0) * C1 / (a1 * a1) + (ph[1].gamma - 1.0) * C2 / (a2 * a2);
}

void orc_heat_capacity(const orc_grid* g, const orc_phase ph[2], double eps, const double* alpha2,
                       const double* m1, const double* m2, const double* T, double* C) {
    int64_t N = ncells(g);
    double B1 = ph[0].pinf - ph[1].pinf;
    for (int64_t i = 0; i < N; ++i) {
        double C1 = m1[i] * ph[0].cv, C2 = m2[i] * ph[1].cv;
        double c = C1 + C2;
        if (B1 != 0.0 && is_mixed(alpha2[i], eps)) {
            double W = pressure_stiffness(ph, alpha2[i], C1, C2);
            c += B1 * B1 / (T[i] * T[i] * W);
        }
        C[i] = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Discrete operator D v = -div(Lambda grad v) (eq. qk_dis, all axes).       */
/* Every loop below visits cells (i,j,k) independently; the (k,j) rows are  */
/* shared out over OpenMP threads, which changes no arithmetic.              */

double orc_gershgorin(const orc_grid* g, const double* Lam, const double* C,
                      const double axis_scale[3], int32_t face_mean) {
    double lam = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(max : lam)
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t a = i + g->n[0] * (j + g->n[1] * k);
                cell_faces f;
                faces_of(g, axis_scale, i, j, k, &f);
                /* d_a = sum_f w_f Lambda_f / C_a: the diagonal of A, equal to the
                 * sum of the magnitudes of the off-diagonal entries of row a. */
                double d = 0.0;
                for (int q = 0; q < f.count; ++q) d += f.w[q] * face_value(Lam[a], Lam[f.nb[q]], face_mean);
                double r = 2.0 * d / C[a];
                if (r > lam) lam = r;
            }
    return lam;
}

/* div[a] = sum over faces of a of w Lambda_f (v_nb - v_a): the net flux into a.
 * The flux through a face is the same number seen from either side, with
 * opposite sign, so the sum over all cells cancels face by face. */
static void face_flux_divergence(const orc_grid* g, const double* Lam, const double axis_scale[3],
                                 int32_t face_mean, const double* v, double* div) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t a = i + g->n[0] * (j + g->n[1] * k);
                cell_faces f;
                faces_of(g, axis_scale, i, j, k, &f);
                double s = 0.0;
                for (int q = 0; q < f.count; ++q) {
                    int64_t b = f.nb[q];
                    s += f.w[q] * face_value(Lam[a], Lam[b], face_mean) * (v[b] - v[a]);
                }
                div[a] = s;
            }
}

void orc_apply_A(const orc_grid* g, const double* Lam, const double* C, const double axis_scale[3],
                 int32_t face_mean, const double* v, double* y) {
    int64_t N = ncells(g);
    face_flux_divergence(g, Lam, axis_scale, face_mean, v, y);
    for (int64_t a = 0; a < N; ++a) y[a] = -y[a] / C[a];
}

/* ------------------------------------------------------------------------ */
/* Method of local iterations (Sec. 3.2, eqs. LIM and LIM_last).              */

void orc_lim_pass(const orc_grid* g, const double* Lam, const double* C, const double axis_scale[3],
                  int32_t face_mean, double tau, int32_t nst, const double* b, const double* rhs,
                  const double* v0, double* out, double* stages) {
    int64_t N = ncells(g);
    double* cur = dalloc(N);
    double* nxt = dalloc(N);
    double* Av = dalloc(N);
    memcpy(cur, v0, sizeof(double) * (size_t)N);
    /* stages 1 .. nst-1: v^(m) = (g + tau b_m v^(m-1) - tau A v^(m-1)) / (1 + tau b_m) */
    for (int32_t m = 1; m < nst; ++m) {
        if (stages) memcpy(stages + (int64_t)(m - 1) * N, cur, sizeof(double) * (size_t)N);
        orc_apply_A(g, Lam, C, axis_scale, face_mean, cur, Av);
        double tb = tau * b[m - 1];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) nxt[i] = (rhs[i] + tb * cur[i] - tau * Av[i]) / (1.0 + tb);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (stages) memcpy(stages + (int64_t)(nst - 1) * N, cur, sizeof(double) * (size_t)N);
    /* last stage, b = 0: conservative flux difference of the predicted v_hat */
    face_flux_divergence(g, Lam, axis_scale, face_mean, cur, Av);
    for (int64_t i = 0; i < N; ++i) out[i] = rhs[i] + tau * Av[i] / C[i];
    free(cur);
    free(nxt);
    free(Av);
}

double orc_be_residual(const orc_grid* g, const double* Lam, const double* C,
                       const double axis_scale[3], int32_t face_mean, double tau, const double* rhs,
                       const double* v) {
    int64_t N = ncells(g);
    double* div = dalloc(N);
    face_flux_divergence(g, Lam, axis_scale, face_mean, v, div);
    double rr = 0.0, gg = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        /* C (g - v) - tau D v, with D v = -div */
        double r = C[i] * (rhs[i] - v[i]) + tau * div[i];
        rr += r * r;
        gg += (C[i] * rhs[i]) * (C[i] * rhs[i]);
    }
    free(div);
    return gg > 0.0 ? sqrt(rr / gg) : sqrt(rr);
}

/* Chebyshev-Richardson cycles of s stages towards (I + tau A) v = g. */
int32_t orc_cycle_solve(const orc_grid* g, const double* Lam, const double* C,
                        const double axis_scale[3], int32_t face_mean, double tau,
                        double lambda_max, int32_t s, const double* rhs, const double* v0,
                        double tol, int32_t max_cycles, double* out, double* residual_hist) {
    int64_t N = ncells(g);
    double* b = dalloc(s);
    double* Av = dalloc(N);
    orc_cycle_params(s, lambda_max, b);
    memcpy(out, v0, sizeof(double) * (size_t)N);
    int32_t cyc = 0;
    while (cyc < max_cycles) {
        for (int32_t m = 0; m < s; ++m) {
            orc_apply_A(g, Lam, C, axis_scale, face_mean, out, Av);
            double tb = tau * b[m];
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) out[i] = (rhs[i] + tb * out[i] - tau * Av[i]) / (1.0 + tb);
        }
        ++cyc;
        double r = orc_be_residual(g, Lam, C, axis_scale, face_mean, tau, rhs, out);
        if (residual_hist) residual_hist[cyc - 1] = r;
        if (r < tol) break;
    }
    free(b);
    free(Av);
    return cyc;
}

/* ------------------------------------------------------------------------ */
/* Temperature relaxation (Sec. 3.4.1).                                      */

/* Sign of p_1 - p_2 at alpha_2 = a, times a(1-a) > 0, with T(a) from the
 * energy balance.  Returned as the quadratic T(a)(G1 C1 a - G2 C2 (1-a)) + B a (1-a). */
static double relax_pressure_gap(const orc_phase ph[2], double C1, double C2, double Esens,
                                 double a20, double a) {
    double B = ph[1].pinf - ph[0].pinf;
    double T = (Esens + (a20 - a) * B) / (C1 + C2);
    return T * ((ph[0].gamma - 1.0) * C1 * a - (ph[1].gamma - 1.0) * C2 * (1.0 - a)) + B * a * (1.0 - a);
}

void orc_relax(const orc_grid* g, const orc_phase ph[2], double eps, double* alpha2,
               const double* m1, const double* m2, double* T1, double* T2) {
    int64_t N = ncells(g);
    double B = ph[1].pinf - ph[0].pinf; /* p_inf,2 - p_inf,1 */
    for (int64_t i = 0; i < N; ++i) {
        double a20 = alpha2[i];
        if (a20 <= eps) { /* only phase 1 present */
            T2[i] = T1[i];
            continue;
        }
        if (a20 >= 1.0 - eps) { /* only phase 2 present */
            T1[i] = T2[i];
            continue;
        }
        double C1 = m1[i] * ph[0].cv, C2 = m2[i] * ph[1].cv;
        /* Energy: sum_k C_k T_k + alpha_k p_inf,k is conserved, so
         * (C1 + C2) T'(a) = C1 T1 + C2 T2 + (alpha2^0 - a) B. */
        double Esens = C1 * T1[i] + C2 * T2[i];
        /* Admissible interval: 0 < a < 1 and T'(a) > 0. */
        double lo = 0.0, hi = 1.0;
        if (B > 0.0) {
            double lim = a20 + Esens / B;
            if (lim < hi) hi = lim;
        } else if (B < 0.0) {
            double lim = a20 + Esens / B;
            if (lim > lo) lo = lim;
        }
        /* p_1 - p_2 goes from -inf (or -|B|) at lo to +inf (or +B) at hi and has
         * a single root there: plain bisection. */
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (relax_pressure_gap(ph, C1, C2, Esens, a20, mid) < 0.0) lo = mid;
            else hi = mid;
        }
        double a = 0.5 * (lo + hi);
        double T = (Esens + (a20 - a) * B) / (C1 + C2);
        alpha2[i] = a;
        T1[i] = T;
        T2[i] = T;
    }
}

double orc_energy(const orc_grid* g, const orc_phase ph[2], const double* alpha2, const double* m1,
                  const double* m2, const double* T1, const double* T2) {
    int64_t N = ncells(g);
    double e = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double a2 = alpha2[i], a1 = 1.0 - a2;
        e += m1[i] * ph[0].cv * T1[i] + m2[i] * ph[1].cv * T2[i] + a1 * ph[0].pinf + a2 * ph[1].pinf;
    }
    return e * cell_volume(g);
}

/* ------------------------------------------------------------------------ */
/* Picard loop of Algorithm 1 around LIM passes (no relaxation inside).       */

static const double UNIT_SCALE[3] = {1.0, 1.0, 1.0};

/* Heat conduction for one step from the relaxed state (alpha2, T).
 * T holds T^n on entry and T^{n+1} on exit; alpha2 likewise. */
static int32_t heat_picard(const orc_grid* g, const orc_phase ph[2], const orc_opts* o,
                           double* alpha2, const double* m1, const double* m2, double* T,
                           const double* src1, const double* src2, const double* frozen_lambda,
                           double* E, orc_report* rep) {
    int64_t N = ncells(g);
    double tau = o->tau;
    double B1 = ph[0].pinf - ph[1].pinf;
    double* Tn = dalloc(N);
    double* a2n = dalloc(N);
    double* Lam = dalloc(N);
    double* C = dalloc(N);
    double* rhs = dalloc(N);
    double* Tnew = dalloc(N);
    memcpy(Tn, T, sizeof(double) * (size_t)N);
    memcpy(a2n, alpha2, sizeof(double) * (size_t)N);
    int32_t converged = 0, it;
    for (it = 0; it < o->passes; ++it) {
        /* Coefficients lagged at T^(it), alpha2^(it). */
        orc_cell_conductivity(g, ph, alpha2, m1, m2, T, Lam);
        orc_heat_capacity(g, ph, o->alpha_eps, alpha2, m1, m2, T, C);
        for (int64_t i = 0; i < N; ++i) {
            double f = 0.0;
            if (src1) f += (1.0 - alpha2[i]) * src1[i];
            if (src2) f += alpha2[i] * src2[i];
            rhs[i] = Tn[i] + tau * f / C[i];
        }
        double lam = frozen_lambda ? frozen_lambda[it]
                                   : orc_gershgorin(g, Lam, C, UNIT_SCALE, o->face_mean);
        int32_t P = orc_lim_P(tau, lam);
        int32_t nst = 2 * P - 1;
        if (o->cycle_mode) {
            double res = 0.0;
            double* hist = dalloc(o->max_cycles > 0 ? o->max_cycles : 1);
            int32_t nc = orc_cycle_solve(g, Lam, C, UNIT_SCALE, o->face_mean, tau, lam, nst, rhs, Tn,
                                         o->cycle_tol, o->max_cycles, Tnew, hist);
            res = nc > 0 ? hist[nc - 1] : 0.0;
            free(hist);
            if (rep && it < ORC_MAX_PASSES) {
                rep->cycles[it] = nc;
                rep->residual[it] = res;
            }
        } else {
            double* b = dalloc(nst);
            orc_lim_params(P, lam, o->order, b);
            orc_lim_pass(g, Lam, C, UNIT_SCALE, o->face_mean, tau, nst, b, rhs, Tn, Tnew, NULL);
            free(b);
        }
        /* Volume fraction (Algorithm 1, second solve): d alpha2 = -B1/(T^2 W) dT,
         * integrated from the step start with the lagged coefficient. */
        if (B1 != 0.0) {
            for (int64_t i = 0; i < N; ++i) {
                if (!is_mixed(a2n[i], o->alpha_eps)) continue;
                double C1 = m1[i] * ph[0].cv, C2 = m2[i] * ph[1].cv;
                double W = pressure_stiffness(ph, alpha2[i], C1, C2);
                alpha2[i] = a2n[i] - B1 / (T[i] * T[i] * W) * (Tnew[i] - Tn[i]);
            }
        }
        double dmax = 0.0, tmax = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double d = fabs(Tnew[i] - T[i]);
            if (d > dmax) dmax = d;
            if (fabs(Tnew[i]) > tmax) tmax = fabs(Tnew[i]);
        }
        double err = tmax > 0.0 ? dmax / tmax : dmax;
        memcpy(T, Tnew, sizeof(double) * (size_t)N);
        if (rep && it < ORC_MAX_PASSES) {
            rep->P[it] = P;
            rep->lambda_G[it] = lam;
            rep->err[it] = err;
        }
        if (o->picard_tol > 0.0 && err < o->picard_tol) {
            converged = 1;
            ++it;
            break;
        }
    }
    if (rep) {
        rep->passes_run = it;
        rep->converged = converged || o->picard_tol <= 0.0;
    }
    /* Total energy: the last pass's final stage moved C_eff (T^{n+1} - T^n)
     * into each cell, its flux divergence plus sources. */
    if (E)
        for (int64_t i = 0; i < N; ++i) E[i] += C[i] * (T[i] - Tn[i]);
    free(Tn);
    free(a2n);
    free(Lam);
    free(C);
    free(rhs);
    free(Tnew);
    return (o->picard_tol > 0.0 && !converged) ? 3 : 0;
}

/* Viscous heating (Sec. 3.2, phase internal energies).  Along axis d the
 * viscous flux through the face between cell a and b = a + e_d is
 * F = s_d mu_f (uh_b - uh_a) / h_d, with face values uh_f = (uh_a + uh_b)/2
 * and alpha_k,f = (alpha_k,a + alpha_k,b)/2.  The energy of phase k in cell a
 * changes by
 *   tau/h_d [alpha_k,f+ uh_f+ F_f+ - alpha_k,f- uh_f- F_f-]
 *     - tau/h_d uh_a [alpha_k,f+ F_f+ - alpha_k,f- F_f-]
 * summed over the axes (f+ / f- the faces towards a + e_d / a - e_d; a face
 * that does not exist carries no flux).  With rho_k and alpha_k fixed in
 * this part, T_k changes by that energy over C_k = m_k C_v,k; in a cell
 * without phase k (alpha_k outside (eps, 1-eps)) the phase present takes
 * both shares. */
void orc_visc_heat(const orc_grid* g, const orc_phase ph[2], double eps, int32_t face_mean,
                   const double* alpha2, const double* m1, const double* m2, const double* mu,
                   const double axis_scale[3], double tau, const double* uh, double* T1, double* T2) {
    const int64_t stride[3] = {1, g->n[0], g->n[0] * g->n[1]};
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                const int64_t c[3] = {i, j, k};
                const int64_t a = i + g->n[0] * (j + g->n[1] * k);
                double dE[2] = {0.0, 0.0};
                for (int axis = 0; axis < 3; ++axis) {
                    const int64_t n = g->n[axis];
                    if (n <= 1) continue;
                    const double h = g->h[axis];
                    /* F, uh_f and alpha_k,f of the faces a+e_d (side +1) and a-e_d (side -1) */
                    double F[2] = {0.0, 0.0}, uf[2] = {0.0, 0.0}, af[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
                    for (int side = 0; side < 2; ++side) {
                        const int dir = side == 0 ? 1 : -1;
                        int64_t cn = c[axis] + dir;
                        if (cn < 0 || cn >= n) {
                            if (g->bc[axis] != ORC_PERIODIC) continue;
                            cn = (cn + n) % n;
                        }
                        const int64_t b = a + (cn - c[axis]) * stride[axis];
                        const double muf = face_value(mu[a], mu[b], face_mean);
                        /* flux in the +d direction through this face */
                        const double grad = dir > 0 ? (uh[b] - uh[a]) / h : (uh[a] - uh[b]) / h;
                        F[side] = axis_scale[axis] * muf * grad;
                        uf[side] = 0.5 * (uh[a] + uh[b]);
                        af[side][0] = 0.5 * ((1.0 - alpha2[a]) + (1.0 - alpha2[b]));
                        af[side][1] = 0.5 * (alpha2[a] + alpha2[b]);
                    }
                    for (int ph_k = 0; ph_k < 2; ++ph_k) {
                        const double work = af[0][ph_k] * uf[0] * F[0] - af[1][ph_k] * uf[1] * F[1];
                        const double force = af[0][ph_k] * F[0] - af[1][ph_k] * F[1];
                        dE[ph_k] += tau / h * work - tau / h * uh[a] * force;
                    }
                }
                const double a2 = alpha2[a];
                const double C1 = m1[a] * ph[0].cv, C2 = m2[a] * ph[1].cv;
                if (a2 <= eps) {
                    T1[a] += (dE[0] + dE[1]) / C1;
                } else if (a2 >= 1.0 - eps) {
                    T2[a] += (dE[0] + dE[1]) / C2;
                } else {
                    T1[a] += dE[0] / C1;
                    T2[a] += dE[1] / C2;
                }
            }
}

/* Total-energy update of the viscous part (Sec. 3.2): the divergence of the
 * work uh_f F_f of the viscous flux, face by face as in orc_visc_heat. */
void orc_visc_energy(const orc_grid* g, int32_t face_mean, const double* mu, const double axis_scale[3],
                     double tau, const double* uh, double* E) {
    const int64_t stride[3] = {1, g->n[0], g->n[0] * g->n[1]};
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                const int64_t c[3] = {i, j, k};
                const int64_t a = i + g->n[0] * (j + g->n[1] * k);
                double dE = 0.0;
                for (int axis = 0; axis < 3; ++axis) {
                    const int64_t n = g->n[axis];
                    if (n <= 1) continue;
                    const double h = g->h[axis];
                    double work[2] = {0.0, 0.0}; /* uh_f F_f at the faces a+e_d, a-e_d */
                    for (int side = 0; side < 2; ++side) {
                        const int dir = side == 0 ? 1 : -1;
                        int64_t cn = c[axis] + dir;
                        if (cn < 0 || cn >= n) {
                            if (g->bc[axis] != ORC_PERIODIC) continue;
                            cn = (cn + n) % n;
                        }
                        const int64_t b = a + (cn - c[axis]) * stride[axis];
                        const double muf = face_value(mu[a], mu[b], face_mean);
                        const double grad = dir > 0 ? (uh[b] - uh[a]) / h : (uh[a] - uh[b]) / h;
                        work[side] = 0.5 * (uh[a] + uh[b]) * axis_scale[axis] * muf * grad;
                    }
                    dE += tau / h * (work[0] - work[1]);
                }
                E[a] += dE;
            }
}

/* Viscous momentum diffusion, one LIM pass per velocity component, with the
 * viscous heating of the phases and the total-energy update when asked. */
static void viscous(const orc_grid* g, const orc_phase ph[2], const orc_opts* o,
                    const double* alpha2, const double* m1, const double* m2, double* vel[3],
                    const double* frozen_visc, double* T1, double* T2, double* E, orc_report* rep) {
    int64_t N = ncells(g);
    double* rho = dalloc(N);
    double* mu = dalloc(N);
    double* out = dalloc(N);
    for (int64_t i = 0; i < N; ++i) {
        rho[i] = m1[i] + m2[i];
        mu[i] = (1.0 - alpha2[i]) * ph[0].mu + alpha2[i] * ph[1].mu;
    }
    for (int c = 0; c < 3; ++c) {
        if (g->n[c] <= 1 || !vel[c]) continue;
        /* rho du_c/dt = sum_d d_d(mu_cd d_d u_c), mu_cd = 4/3 mu on the own axis. */
        double s[3] = {1.0, 1.0, 1.0};
        s[c] = 4.0 / 3.0;
        double lam = frozen_visc ? frozen_visc[c] : orc_gershgorin(g, mu, rho, s, o->face_mean);
        int32_t P = orc_lim_P(o->tau, lam);
        int32_t nst = 2 * P - 1;
        double* b = dalloc(nst);
        orc_lim_params(P, lam, o->order, b);
        if (o->visc_heating || E) {
            /* keep the stage iterates: the last one, v^(2P-2), is the predicted velocity */
            double* st = dalloc((int64_t)nst * N);
            orc_lim_pass(g, mu, rho, s, o->face_mean, o->tau, nst, b, vel[c], vel[c], out, st);
            const double* uh = st + (int64_t)(nst - 1) * N;
            if (o->visc_heating)
                orc_visc_heat(g, ph, o->alpha_eps, o->face_mean, alpha2, m1, m2, mu, s, o->tau, uh, T1, T2);
            if (E) orc_visc_energy(g, o->face_mean, mu, s, o->tau, uh, E);
            free(st);
        } else {
            orc_lim_pass(g, mu, rho, s, o->face_mean, o->tau, nst, b, vel[c], vel[c], out, NULL);
        }
        memcpy(vel[c], out, sizeof(double) * (size_t)N);
        free(b);
        if (rep) {
            rep->visc_P[c] = P;
            rep->visc_lambda_G[c] = lam;
        }
    }
    free(rho);
    free(mu);
    free(out);
}

int32_t orc_step(const orc_grid* g, const orc_phase ph[2], const orc_opts* o, double* alpha2,
                 const double* m1, const double* m2, double* T1, double* T2, const double* src1,
                 const double* src2, double* u, double* v, double* w, double* E, const double* frozen_lambda,
                 const double* frozen_visc, orc_report* rep) {
    if (rep) memset(rep, 0, sizeof(*rep));
    if (rep) rep->energy_before = orc_energy(g, ph, alpha2, m1, m2, T1, T2);
    /* Splitting order of the paper: viscous part, then temperature relaxation,
     * then heat conduction. */
    if (o->do_viscous) {
        double* vel[3] = {u, v, w};
        viscous(g, ph, o, alpha2, m1, m2, vel, frozen_visc, T1, T2, E, rep);
    }
    orc_relax(g, ph, o->alpha_eps, alpha2, m1, m2, T1, T2);
    int32_t st = heat_picard(g, ph, o, alpha2, m1, m2, T1, src1, src2, frozen_lambda, E, rep);
    memcpy(T2, T1, sizeof(double) * (size_t)ncells(g));
    if (rep) rep->energy_after = orc_energy(g, ph, alpha2, m1, m2, T1, T2);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the heat steps (discrete reverse of the LIM passes).           */

/* Reverse of one LIM pass.  stages holds v^(0..nst-1); lam_io holds dL/dv^(nst)
 * on entry and dL/dv^(0) on exit; dL/dg is added to dg and dL/dLambda_cell
 * (through the face means) to gLam. */
static void lim_pass_reverse(const orc_grid* g, const double* Lam, const double* C,
                             const double axis_scale[3], int32_t face_mean, double tau, int32_t nst,
                             const double* b, const double* stages, double* lam_io, double* dg,
                             double* gLam) {
    int64_t N = ncells(g);
    double* wv = dalloc(N);
    double* div = dalloc(N);
    for (int32_t m = nst; m >= 1; --m) {
        double tb = tau * b[m - 1];
        double cm = 1.0 / (1.0 + tb);
        const double* vp = stages + (int64_t)(m - 1) * N;
        for (int64_t i = 0; i < N; ++i) dg[i] += cm * lam_io[i];
        /* Stage m: v^(m)_a = cm (g_a + tb v_a - tau/C_a sum_f w Lambda_f (v_a - v_b)),
         * v = v^(m-1).  Lambda_f enters rows a and b:
         * dL/dLambda_f = cm tau w (v_b - v_a)(lambda_a/C_a - lambda_b/C_b),
         * the same number from either side; each side adds its own share
         * dLambda_f/dLambda_cell. */
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t k = 0; k < g->n[2]; ++k)
            for (int64_t j = 0; j < g->n[1]; ++j)
                for (int64_t i = 0; i < g->n[0]; ++i) {
                    int64_t a = i + g->n[0] * (j + g->n[1] * k);
                    cell_faces f;
                    faces_of(g, axis_scale, i, j, k, &f);
                    double s = 0.0;
                    for (int q = 0; q < f.count; ++q) {
                        int64_t bb = f.nb[q];
                        double G = cm * tau * f.w[q] * (vp[bb] - vp[a]) *
                                   (lam_io[a] / C[a] - lam_io[bb] / C[bb]);
                        s += G * face_partial(Lam[a], Lam[bb], face_mean);
                    }
                    gLam[a] += s;
                }
        /* lambda^(m-1) = cm (tb lambda^(m) - tau D C^-1 lambda^(m)), D w = -div(w):
         * A = C^-1 D with D symmetric, so A^T = D C^-1. */
        for (int64_t i = 0; i < N; ++i) wv[i] = lam_io[i] / C[i];
        face_flux_divergence(g, Lam, axis_scale, face_mean, wv, div);
        for (int64_t i = 0; i < N; ++i) lam_io[i] = cm * (tb * lam_io[i] + tau * div[i]);
    }
    free(wv);
    free(div);
}

int32_t orc_heat_adjoint(const orc_grid* g, const orc_phase ph[2], const orc_opts* o, int32_t nsteps,
                         const double* lamsched, const double* alpha2, const double* m1,
                         const double* m2, const double* T0, const double* dL_dTN, double* dL_dT0,
                         double* dL_dk0, double* TN) {
    if (ph[0].pinf != ph[1].pinf || o->cycle_mode || o->do_viscous) return 1;
    int64_t N = ncells(g);
    int32_t np = o->passes;
    double tau = o->tau;
    double* C = dalloc(N);
    double* Lam = dalloc(N);
    double* Tsteps = dalloc(N * (nsteps + 1));
    double* Tpass = dalloc(N * (np + 1));
    double* mu = dalloc(N);
    double* acc = dalloc(N);
    double* dg = dalloc(N);
    double* gLam = dalloc(N);
    int32_t Pmax = 1;
    for (int32_t k = 0; k < nsteps * np; ++k) {
        int32_t P = orc_lim_P(tau, lamsched[k]);
        if (P > Pmax) Pmax = P;
    }
    int64_t stride = (int64_t)(2 * Pmax - 1) * N;
    double* stages = dalloc(stride * np);
    double* b = dalloc(2 * Pmax - 1);
    /* alpha2 is frozen and C constant when p_inf,1 = p_inf,2. */
    orc_heat_capacity(g, ph, o->alpha_eps, alpha2, m1, m2, T0, C);

    /* Forward sweep, keeping T^n of every step. */
    memcpy(Tsteps, T0, sizeof(double) * (size_t)N);
    for (int32_t n = 0; n < nsteps; ++n) {
        const double* Tn = Tsteps + (int64_t)n * N;
        memcpy(Tpass, Tn, sizeof(double) * (size_t)N);
        for (int32_t it = 0; it < np; ++it) {
            double lam = lamsched[n * np + it];
            int32_t P = orc_lim_P(tau, lam), nst = 2 * P - 1;
            orc_lim_params(P, lam, o->order, b);
            orc_cell_conductivity(g, ph, alpha2, m1, m2, Tpass + (int64_t)it * N, Lam);
            orc_lim_pass(g, Lam, C, UNIT_SCALE, o->face_mean, tau, nst, b, Tn, Tn,
                         Tpass + (int64_t)(it + 1) * N, NULL);
        }
        memcpy(Tsteps + (int64_t)(n + 1) * N, Tpass + (int64_t)np * N, sizeof(double) * (size_t)N);
    }
    if (TN) memcpy(TN, Tsteps + (int64_t)nsteps * N, sizeof(double) * (size_t)N);

    /* Reverse sweep. */
    memcpy(mu, dL_dTN, sizeof(double) * (size_t)N);
    dL_dk0[0] = dL_dk0[1] = 0.0;
    for (int32_t n = nsteps - 1; n >= 0; --n) {
        const double* Tn = Tsteps + (int64_t)n * N;
        /* Recompute the passes of this step, keeping T^(it) and every stage. */
        memcpy(Tpass, Tn, sizeof(double) * (size_t)N);
        for (int32_t it = 0; it < np; ++it) {
            double lam = lamsched[n * np + it];
            int32_t P = orc_lim_P(tau, lam), nst = 2 * P - 1;
            orc_lim_params(P, lam, o->order, b);
            orc_cell_conductivity(g, ph, alpha2, m1, m2, Tpass + (int64_t)it * N, Lam);
            orc_lim_pass(g, Lam, C, UNIT_SCALE, o->face_mean, tau, nst, b, Tn, Tn,
                         Tpass + (int64_t)(it + 1) * N, stages + it * stride);
        }
        /* mu = dL/dT^{n+1}, the adjoint of the last pass's output; acc collects dL/dT^n. */
        memset(acc, 0, sizeof(double) * (size_t)N);
        for (int32_t it = np - 1; it >= 0; --it) {
            double lam = lamsched[n * np + it];
            int32_t P = orc_lim_P(tau, lam), nst = 2 * P - 1;
            orc_lim_params(P, lam, o->order, b);
            const double* Tit = Tpass + (int64_t)it * N;
            orc_cell_conductivity(g, ph, alpha2, m1, m2, Tit, Lam);
            memset(dg, 0, sizeof(double) * (size_t)N);
            memset(gLam, 0, sizeof(double) * (size_t)N);
            lim_pass_reverse(g, Lam, C, UNIT_SCALE, o->face_mean, tau, nst, b, stages + it * stride,
                             mu, dg, gLam);
            /* The pass reads T^n twice: as g and as v^(0). */
            for (int64_t i = 0; i < N; ++i) acc[i] += dg[i] + mu[i];
            /* Lambda_i = sum_k alpha_k lambda_k(rho_i, T_i), evaluated at T^(it);
             * lambda_k is proportional to k0_k. */
            for (int64_t i = 0; i < N; ++i) {
                double a2 = alpha2[i], a1 = 1.0 - a2, rho = m1[i] + m2[i];
                dL_dk0[0] += gLam[i] * a1 * conductivity_per_k0(&ph[0], Tit[i], rho);
                dL_dk0[1] += gLam[i] * a2 * conductivity_per_k0(&ph[1], Tit[i], rho);
                mu[i] = gLam[i] * (a1 * conductivity_dT(&ph[0], Tit[i], rho) +
                                   a2 * conductivity_dT(&ph[1], Tit[i], rho));
            }
            /* T^(1) = T^n, so the first pass's coefficient gradient is T^n's;
             * otherwise mu is the adjoint of the previous pass's output. */
            if (it == 0)
                for (int64_t i = 0; i < N; ++i) acc[i] += mu[i];
        }
        memcpy(mu, acc, sizeof(double) * (size_t)N);
    }
    memcpy(dL_dT0, mu, sizeof(double) * (size_t)N);
    free(C);
    free(Lam);
    free(Tsteps);
    free(Tpass);
    free(mu);
    free(acc);
    free(dg);
    free(gLam);
    free(stages);
    free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Hyperbolic part and pressure relaxation (Sec. 3.1 and Sec. 3.3).          */
/*                                                                            */
/* Conservative state per cell, in the order of the vector U of eq.           */
/* vectorForm (three momentum components here):                               */
/*   q[0] = alpha_1 rho_1, q[1] = alpha_2 rho_2, q[2..4] = rho u, rho v,      */
/*   rho w, q[5] = alpha_1 rho_1 e_1, q[6] = alpha_2 rho_2 e_2, q[7] = rho E, */
/*   q[8] = alpha_2.                                                          */
/* Phase energies follow the SG EOS (eqs. eos_stiffened, eos_stiffened2):    */
/*   alpha_k rho_k e_k = alpha_k (p_k + gamma_k p_inf,k)/(gamma_k - 1)        */
/*                       + alpha_k rho_k q_k                                   */
/*                     = alpha_k rho_k C_v,k T_k + alpha_k p_inf,k            */
/*                       + alpha_k rho_k q_k.                                 */

#define NQ 9

/* alpha_k p_k of phase k from its partial energy and mass. */
static double phase_alpha_p(const orc_phase* p, double ak, double mk, double Ek) {
    return (p->gamma - 1.0) * (Ek - mk * p->q) - p->gamma * ak * p->pinf;
}

typedef struct {
    double rho, un, p, c;  /* mixture density, normal velocity, pressure, sound speed */
} hyp_prim;

/* Mixture quantities of a state for the normal axis d: p = sum alpha_k p_k,
 * and the speed of sound of the model, c^2 = Y_1 c_1^2 + Y_2 c_2^2 with
 * c_k^2 = gamma_k (p_k + p_inf,k)/rho_k (so rho c^2 = sum gamma_k alpha_k
 * (p_k + p_inf,k)). */
static hyp_prim hyp_mixture(const orc_phase ph[2], const double* q, int d) {
    hyp_prim s;
    double a2 = q[8], a1 = 1.0 - a2;
    s.rho = q[0] + q[1];
    s.un = q[2 + d] / s.rho;
    double ap1 = phase_alpha_p(&ph[0], a1, q[0], q[5]);
    double ap2 = phase_alpha_p(&ph[1], a2, q[1], q[6]);
    s.p = ap1 + ap2;
    double rc2 = ph[0].gamma * (ap1 + a1 * ph[0].pinf) + ph[1].gamma * (ap2 + a2 * ph[1].pinf);
    s.c = sqrt(rc2 / s.rho);
    return s;
}

/* HLLC solution at a face between states L and R along axis d (Sec. 3.1;
 * three-wave solver with Davis speed estimates).  Returns the face flux of
 * every component as in eq. vectorForm, F = u U + p D (D has 1 in the normal
 * momentum and u in rho E), and the face velocity u* used by the
 * non-conservative terms R(U) du/dx.  Star states: every advected density is
 * scaled by (S_K - u_K)/(S_K - S*) -- the phase masses, the tangential
 * momenta and the phase internal energies (their specific values carried
 * across the waves) -- alpha_2 is continuous across S_K, the normal momentum
 * is rho* S*, and the total energy takes the HLLC jump. */
static void hllc_face(const orc_phase ph[2], const double* qL, const double* qR, int d, double* F,
                      double* ustar) {
    hyp_prim L = hyp_mixture(ph, qL, d), R = hyp_mixture(ph, qR, d);
    double SL = fmin(L.un - L.c, R.un - R.c);
    double SR = fmax(L.un + L.c, R.un + R.c);
    double Ss = (R.p - L.p + L.rho * L.un * (SL - L.un) - R.rho * R.un * (SR - R.un)) /
                (L.rho * (SL - L.un) - R.rho * (SR - R.un));
    double U[NQ];
    double uf, pf;
    if (SL >= 0.0) {
        memcpy(U, qL, sizeof(U));
        uf = L.un;
        pf = L.p;
    } else if (SR <= 0.0) {
        memcpy(U, qR, sizeof(U));
        uf = R.un;
        pf = R.p;
    } else {
        const double* qK = Ss >= 0.0 ? qL : qR;
        const hyp_prim* K = Ss >= 0.0 ? &L : &R;
        double SK = Ss >= 0.0 ? SL : SR;
        double f = (SK - K->un) / (SK - Ss);
        for (int c = 0; c < NQ; ++c) U[c] = qK[c] * f;
        U[2 + d] = K->rho * f * Ss;
        U[7] = f * (qK[7] + (Ss - K->un) * (K->rho * Ss + K->p / (SK - K->un)));
        U[8] = qK[8];
        uf = Ss;
        pf = K->p + K->rho * (SK - K->un) * (Ss - K->un);
    }
    for (int c = 0; c < NQ; ++c) F[c] = uf * U[c];
    F[2 + d] += pf;
    F[7] += pf * uf;
    *ustar = uf;
}

/* Ghost state behind a wall at the end of axis d: the mirror image of the
 * boundary cell (normal momentum reversed). */
static void wall_ghost(const double* q, int d, double* g) {
    memcpy(g, q, sizeof(double) * NQ);
    g[2 + d] = -q[2 + d];
}

/* One Godunov sweep along axis d (eq. of the Godunov method in Sec. 3.1):
 * U_i -= dt/h (F_{i+1/2} - F_{i-1/2}) + dt/h R(U_i) (u*_{i+1/2} - u*_{i-1/2}),
 * R = (0, 0, 0, 0, 0, alpha_1 p_1, alpha_2 p_2, 0, -alpha_2). */
static void godunov_sweep(const orc_grid* g, const orc_phase ph[2], double dt, int d, double* q[NQ]) {
    int64_t N = ncells(g);
    int64_t n = g->n[d];
    int64_t stride = d == 0 ? 1 : (d == 1 ? g->n[0] : g->n[0] * g->n[1]);
    double lam = dt / g->h[d];
    double* out = dalloc(N * NQ);
    for (int64_t i = 0; i < N; ++i) {
        int64_t pos = (i / stride) % n;
        double qc[NQ], qm[NQ], qp[NQ];
        for (int c = 0; c < NQ; ++c) qc[c] = q[c][i];
        /* left neighbour */
        if (pos > 0 || g->bc[d] == ORC_PERIODIC) {
            int64_t j = pos > 0 ? i - stride : i + (n - 1) * stride;
            for (int c = 0; c < NQ; ++c) qm[c] = q[c][j];
        } else {
            wall_ghost(qc, d, qm);
        }
        if (pos < n - 1 || g->bc[d] == ORC_PERIODIC) {
            int64_t j = pos < n - 1 ? i + stride : i - (n - 1) * stride;
            for (int c = 0; c < NQ; ++c) qp[c] = q[c][j];
        } else {
            wall_ghost(qc, d, qp);
        }
        double Fm[NQ], Fp[NQ], um, up;
        hllc_face(ph, qm, qc, d, Fm, &um);
        hllc_face(ph, qc, qp, d, Fp, &up);
        double a2 = qc[8], a1 = 1.0 - a2;
        double R[NQ] = {0.0, 0.0, 0.0, 0.0, 0.0, phase_alpha_p(&ph[0], a1, qc[0], qc[5]),
                        phase_alpha_p(&ph[1], a2, qc[1], qc[6]), 0.0, -a2};
        for (int c = 0; c < NQ; ++c) out[c * N + i] = qc[c] - lam * (Fp[c] - Fm[c]) - lam * R[c] * (up - um);
    }
    for (int c = 0; c < NQ; ++c) memcpy(q[c], out + c * N, sizeof(double) * (size_t)N);
    free(out);
}

/* Saturation condition of the pressure relaxation (Sec. 3.3, step 1): with
 * the phase masses fixed and d(alpha_k rho_k e_k) = -p d alpha_k integrated
 * at the relaxed pressure p, the SG EOS gives
 *   alpha_k(p) = (gamma_k - 1)(E_k^0 - m_k q_k + p alpha_k^0) / (gamma_k (p + p_inf,k)),
 * and p solves alpha_1(p) + alpha_2(p) = 1. */
static double relaxed_alpha(const orc_phase* p, double a0, double m, double E0, double pr) {
    return (p->gamma - 1.0) * (E0 - m * p->q + pr * a0) / (p->gamma * (pr + p->pinf));
}

void orc_pressure_relax_cell(const orc_phase ph[2], double* q) {
    double a20 = q[8], a10 = 1.0 - a20;
    /* sum_k alpha_k(p) - 1 falls from +inf just above -min p_inf,k to below 0:
     * bracket it and bisect. */
    double lo = -fmin(ph[0].pinf, ph[1].pinf);
    double hi = fabs(lo) + 1.0;
    for (int it = 0; it < 2000; ++it) {
        double s = relaxed_alpha(&ph[0], a10, q[0], q[5], hi) + relaxed_alpha(&ph[1], a20, q[1], q[6], hi);
        if (s < 1.0) break;
        hi = 2.0 * hi;
    }
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double s = relaxed_alpha(&ph[0], a10, q[0], q[5], mid) + relaxed_alpha(&ph[1], a20, q[1], q[6], mid);
        if (s > 1.0) lo = mid;
        else hi = mid;
    }
    double p1 = 0.5 * (lo + hi);
    double a1 = relaxed_alpha(&ph[0], a10, q[0], q[5], p1);
    double a2 = 1.0 - a1;
    /* Step 2: the pressure from the mixture energy rho e = rho E - rho |u|^2/2
     * at the relaxed volume fractions (SG mixture), so that energy is
     * conserved.  Step 3: the phase energies at that pressure. */
    double rho = q[0] + q[1];
    double ke = 0.5 * (q[2] * q[2] + q[3] * q[3] + q[4] * q[4]) / rho;
    double rhoe = q[7] - ke;
    double num = rhoe - q[0] * ph[0].q - q[1] * ph[1].q - a1 * ph[0].gamma * ph[0].pinf / (ph[0].gamma - 1.0) -
                 a2 * ph[1].gamma * ph[1].pinf / (ph[1].gamma - 1.0);
    double den = a1 / (ph[0].gamma - 1.0) + a2 / (ph[1].gamma - 1.0);
    double p2 = num / den;
    q[5] = a1 * (p2 + ph[0].gamma * ph[0].pinf) / (ph[0].gamma - 1.0) + q[0] * ph[0].q;
    q[6] = a2 * (p2 + ph[1].gamma * ph[1].pinf) / (ph[1].gamma - 1.0) + q[1] * ph[1].q;
    q[8] = a2;
}

/* State of the library (alpha_2, m_k, T_k, velocity, rho E) <-> U. */
static void hyp_to_cons(const orc_phase ph[2], double a2, double m1, double m2, double T1, double T2,
                        double u, double v, double w, const double* E, double* q) {
    double a1 = 1.0 - a2;
    q[0] = m1;
    q[1] = m2;
    double rho = m1 + m2;
    q[2] = rho * u;
    q[3] = rho * v;
    q[4] = rho * w;
    q[5] = m1 * (ph[0].cv * T1 + ph[0].q) + a1 * ph[0].pinf;
    q[6] = m2 * (ph[1].cv * T2 + ph[1].q) + a2 * ph[1].pinf;
    q[7] = E ? *E : q[5] + q[6] + 0.5 * rho * (u * u + v * v + w * w);
    q[8] = a2;
}

int32_t orc_hyperbolic(const orc_grid* g, const orc_phase ph[2], double dt, int32_t relax_pressure,
                       double* alpha2, double* m1, double* m2, double* T1, double* T2, double* u, double* v,
                       double* w, double* E) {
    int64_t N = ncells(g);
    double* q[NQ];
    for (int c = 0; c < NQ; ++c) q[c] = dalloc(N);
    for (int64_t i = 0; i < N; ++i) {
        double s[NQ];
        hyp_to_cons(ph, alpha2[i], m1[i], m2[i], T1[i], T2[i], u ? u[i] : 0.0, v ? v[i] : 0.0, w ? w[i] : 0.0,
                    E ? E + i : NULL, s);
        for (int c = 0; c < NQ; ++c) q[c][i] = s[c];
    }
    /* Dimensional splitting: each directional sweep is followed by the
     * pressure relaxation, so that every sweep starts from phase energies in
     * pressure equilibrium and consistent with rho E. */
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] <= 1) continue;
        godunov_sweep(g, ph, dt, d, q);
        if (!relax_pressure) continue;
        for (int64_t i = 0; i < N; ++i) {
            double s[NQ];
            for (int c = 0; c < NQ; ++c) s[c] = q[c][i];
            orc_pressure_relax_cell(ph, s);
            for (int c = 0; c < NQ; ++c) q[c][i] = s[c];
        }
    }
    int32_t bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        double s[NQ];
        for (int c = 0; c < NQ; ++c) s[c] = q[c][i];
        double a2 = s[8], a1 = 1.0 - a2, rho = s[0] + s[1];
        alpha2[i] = a2;
        m1[i] = s[0];
        m2[i] = s[1];
        /* T_k from eq. eos_stiffened2 */
        T1[i] = (s[5] - s[0] * ph[0].q - a1 * ph[0].pinf) / (s[0] * ph[0].cv);
        T2[i] = (s[6] - s[1] * ph[1].q - a2 * ph[1].pinf) / (s[1] * ph[1].cv);
        if (u) u[i] = s[2] / rho;
        if (v) v[i] = s[3] / rho;
        if (w) w[i] = s[4] / rho;
        if (E) E[i] = s[7];
        if (!(a2 > 0.0 && a2 < 1.0) || !(T1[i] > 0.0) || !(T2[i] > 0.0)) bad = 1;
    }
    for (int c = 0; c < NQ; ++c) free(q[c]);
    return bad;
}

double orc_hyperbolic_dt(const orc_grid* g, const orc_phase ph[2], double cfl, const double* alpha2,
                         const double* m1, const double* m2, const double* T1, const double* T2, const double* u,
                         const double* v, const double* w) {
    int64_t N = ncells(g);
    double rate = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double s[NQ];
        hyp_to_cons(ph, alpha2[i], m1[i], m2[i], T1[i], T2[i], u ? u[i] : 0.0, v ? v[i] : 0.0, w ? w[i] : 0.0,
                    NULL, s);
        for (int d = 0; d < 3; ++d) {
            if (g->n[d] <= 1) continue;
            hyp_prim m = hyp_mixture(ph, s, d);
            rate = fmax(rate, (fabs(m.un) + m.c) / g->h[d]);
        }
    }
    return rate > 0.0 ? cfl / rate : 0.0;
}
