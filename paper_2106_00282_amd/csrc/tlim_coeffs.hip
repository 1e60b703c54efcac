// Coefficients of a Picard pass and the Gershgorin bound on grids whose heat
// step has no source term (Sec. 3.4.2, eq. qk_dis; bound of eq. LIM).
//
// Per cell: Lambda = sum_k alpha_k lambda_k(T^(it)) and, where it changes,
// 1/C_eff; per cell the bound 2 rC sum_f w_f mean(Lambda_a, Lambda_b), folded
// into a max.  Without sources g = T^n, so no right-hand side is written (the
// stages read T^n), and with p_inf,1 = p_inf,2 the capacity depends on the
// partial densities only, which the parabolic step does not change: 1/C is
// then built by the first pass of a step and read by the others.
//
// The first pass of a step can also take the temperature relaxation
// (Sec. 3.4.1) that precedes it: every strip then relaxes its cells (halo
// rows included) from (alpha2, T1, T2, m1, m2) before building the
// coefficients at the relaxed state, and writes T^n and the relaxed alpha2
// of its own cells to separate arrays (alpha2 is not updated in place, as
// neighbouring strips still read the unrelaxed values of their halo).
//
// One wave owns a strip of 64 columns (62 output columns plus one halo
// column on each side) by kRows rows and marches down it, keeping the
// conductivities of three consecutive rows in registers; the x-neighbours
// come from the adjacent lanes (DPP).  Loads of T and alpha2 are coalesced
// 512 B rows; halo overhead is (kRows+2)/kRows x 64/62.  No LDS, no barrier:
// waves are independent.  Strips of 4 rows: more waves in flight hide the
// memory latency better than the smaller halo of 8 rows saves (the fused
// relaxation kernel measured 23.6 us against 30.2 us at 1024^2).
#include <hip/hip_runtime.h>

#include "tlim_device.h"
#include "tlim_internal.h"

namespace tlim {

namespace {

using phys::cell_conductivity;
using phys::inv_heat_capacity;
using tb::fmean;
using tb::fold;
using tb::from_left;
using tb::from_right;

constexpr int kRows = 4;
constexpr int kOut = 62;
constexpr int kWaves = 4;

struct Coef2DArgs {
    DevPhases ph;
    const double* T;      // T^(it); with relaxation: T1
    const double* T2;     // with relaxation
    double* Tn_out;       // with relaxation: the relaxed T
    double* a2_out;       // with relaxation: the relaxed alpha2
    const double* alpha2;
    const double* m1;
    const double* m2;
    const double* g;      // T^n (read for the FP32 correction source only)
    const double* rC_in;  // 1/C of the step when it is not rebuilt
    double* Lam;          // nullable
    double* rC;           // written when rebuilt
    float* Lam32;         // FP32 contexts
    float* rC32;
    float* q32;
    float* w0;
    double* lam;          // accumulator row of the bound
    int nx, ny, perx, pery;
    double wx, wy, tau, eps;
    int face, rebuild, tiles_x, strips;
    // 3D grids
    int nz, perz, tiles_y, zc;
    double wz;
};

template <bool kRelax, bool kSH>
__global__ void __launch_bounds__(64 * kWaves) k_coeffs2d(Coef2DArgs a) {
    const int lane = threadIdx.x & 63;
    const int strip = tb::xcd_block() * kWaves + (threadIdx.x >> 6);  // strips in XCD order
    if (strip >= a.strips) return;  // wave-uniform
    const int tx = strip % a.tiles_x, ty = strip / a.tiles_x;
    const int xg = tx * kOut - 1 + lane;
    const int xi = fold(xg, a.nx, a.perx);
    const bool out_lane = lane >= 1 && lane <= kOut && xg < a.nx;
    const bool fL = a.perx ? a.nx > 1 : xg > 0;
    const bool fR = a.perx ? a.nx > 1 : xg < a.nx - 1;
    const int y0 = ty * kRows;
    const bool q = a.q32 != nullptr;

    auto at = [&](int y) { return (int64_t)fold(y, a.ny, a.pery) * a.nx + xi; };
    // rows y0-1 .. y0+kRows: T, alpha2 -> Lambda (and g in FP32 contexts).
    // Every word the kernel reads is in flight before the first law
    // evaluation (one round trip to memory, not one per row): m1, m2 for the
    // relaxation, the Spitzer-Harm law and 1/C, and 1/C itself when kept.
    double Lw[kRows + 2], tw[kRows + 2], aw[kRows + 2], gw[kRows + 2];
    double m1w[kRows + 2], m2w[kRows + 2], rcw[kRows + 2];
    const bool need_m = kRelax || kSH || a.rebuild;
    {
        double t2w[kRows + 2];
#pragma unroll
        for (int r = 0; r < kRows + 2; ++r) {
            const int64_t idx = at(y0 - 1 + r);
            tw[r] = a.T[idx];
            aw[r] = a.alpha2[idx];
            if constexpr (kRelax) t2w[r] = a.T2[idx];
            else gw[r] = q ? a.g[idx] : 0.0;
            m1w[r] = need_m ? a.m1[idx] : 0.0;
            m2w[r] = need_m ? a.m2[idx] : 0.0;
            rcw[r] = a.rebuild ? 0.0 : a.rC_in[idx];
        }
        if constexpr (kRelax) {
#pragma unroll
            for (int r = 0; r < kRows + 2; ++r) {
                phys::relax_cell(a.ph, a.eps, aw[r], tw[r], t2w[r], m1w[r], m2w[r], tw[r], aw[r]);
                gw[r] = tw[r];  // g = T^n, the relaxed T
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kRows + 2; ++r) {
        if constexpr (kSH) Lw[r] = phys::cell_conductivity(a.ph, tw[r], aw[r], m1w[r] + m2w[r]);
        else Lw[r] = phys::cell_conductivity_pow(a.ph, tw[r], aw[r]);
    }

    double bound = 0.0;
#pragma unroll
    for (int r = 1; r <= kRows; ++r) {
        const int y = y0 + r - 1;
        const double L = Lw[r], Lm = Lw[r - 1], Lp = Lw[r + 1];
        const double Ll = from_left(L), Lr = from_right(L);
        const float Lf = (float)L;
        const float Llf = from_left(Lf), Lrf = from_right(Lf);
        const double gl = from_left(gw[r]), gr = from_right(gw[r]);
        if (out_lane && y < a.ny) {
            const int64_t o = (int64_t)y * a.nx + xg;
            const bool fD = a.pery ? a.ny > 1 : y > 0;
            const bool fU = a.pery ? a.ny > 1 : y < a.ny - 1;
            if constexpr (kRelax) {
                a.Tn_out[o] = tw[r];
                a.a2_out[o] = aw[r];
            }
            double rc;
            if (a.rebuild) {
                rc = inv_heat_capacity(a.ph, a.eps, tw[r], aw[r], m1w[r], m2w[r]);
                a.rC[o] = rc;
                if (a.rC32) a.rC32[o] = (float)rc;
            } else {
                rc = rcw[r];
            }
            if (a.Lam) a.Lam[o] = L;
            if (a.Lam32) a.Lam32[o] = Lf;
            // faces in the order -x, +x, -y, +y
            double d = 0.0;
            if (fL) d += a.wx * fmean<double>(L, Ll, a.face);
            if (fR) d += a.wx * fmean<double>(L, Lr, a.face);
            if (fD) d += a.wy * fmean<double>(L, Lm, a.face);
            if (fU) d += a.wy * fmean<double>(L, Lp, a.face);
            bound = fmax(bound, 2.0 * d * rc);
            if (q) {
                // q = -tau rC' D' g from the float-rounded Lambda' and rC'
                const double La = (double)Lf, rf = (double)(float)rc, ga = gw[r];
                double S = 0.0;
                if (fL) S += a.wx * fmean<double>(La, (double)Llf, a.face) * (ga - gl);
                if (fR) S += a.wx * fmean<double>(La, (double)Lrf, a.face) * (ga - gr);
                if (fD) S += a.wy * fmean<double>(La, (double)(float)Lm, a.face) * (ga - gw[r - 1]);
                if (fU) S += a.wy * fmean<double>(La, (double)(float)Lp, a.face) * (ga - gw[r + 1]);
                a.q32[o] = (float)(-a.tau * rf * S);
                if (a.w0) a.w0[o] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
    if (lane == 0) {
        const int sl = strip % kSlots;
        atomicMax((unsigned long long*)(a.lam + sl), (unsigned long long)__double_as_longlong(bound + 0.0));
    }
}

// 3D grids: the same per-cell work, with each wave marching through a chunk
// of z planes (kRows3 rows per wave) and keeping the conductivities (and g)
// of the previous, current and next plane in registers.
constexpr int kRows3 = 2;

template <bool kRelax, bool kSH>
__global__ void __launch_bounds__(64 * kWaves) k_coeffs3d(Coef2DArgs a) {
    constexpr int RW = kRows3 + 2;
    const int lane = threadIdx.x & 63;
    // launch order: with the relaxation this kernel measured 8% slower in XCD order
    const int wid = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= a.strips) return;  // wave-uniform
    const int tx = wid % a.tiles_x, rest = wid / a.tiles_x;
    const int ty = rest % a.tiles_y, tz = rest / a.tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int xg = tx * kOut - 1 + lane;
    const int xi = fold(xg, nx, a.perx);
    const bool out_lane = lane >= 1 && lane <= kOut && xg < nx;
    const bool fL = a.perx ? nx > 1 : xg > 0;
    const bool fR = a.perx ? nx > 1 : xg < nx - 1;
    const int y0 = ty * kRows3, z0 = tz * a.zc;
    const int z1 = z0 + a.zc < nz ? z0 + a.zc : nz;
    const bool q = a.q32 != nullptr;

    // 32-bit element offsets (the launcher requires N < 2^32)
    unsigned rowoff[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) rowoff[r] = (unsigned)fold(y0 - 1 + r, ny, a.pery) * (unsigned)nx + (unsigned)xi;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    // T, alpha2 (relaxed when kRelax), Lambda and g of the window rows of plane z
    auto load_plane = [&](int z, double* tw, double* aw, double* Lw, double* gw) {
        const unsigned pz = (unsigned)fold(z, nz, a.perz) * plane;
        // all rows' words in flight before the first law evaluation
        double t2w[RW], m1w[RW], m2w[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const unsigned idx = pz + rowoff[r];
            tw[r] = a.T[idx];
            aw[r] = a.alpha2[idx];
            if constexpr (kRelax) t2w[r] = a.T2[idx];
            else gw[r] = q ? a.g[idx] : 0.0;
            if constexpr (kRelax || kSH) {
                m1w[r] = a.m1[idx];
                m2w[r] = a.m2[idx];
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if constexpr (kRelax) {
                phys::relax_cell(a.ph, a.eps, aw[r], tw[r], t2w[r], m1w[r], m2w[r], tw[r], aw[r]);
                gw[r] = tw[r];
            }
            if constexpr (kSH) Lw[r] = phys::cell_conductivity(a.ph, tw[r], aw[r], m1w[r] + m2w[r]);
            else Lw[r] = phys::cell_conductivity_pow(a.ph, tw[r], aw[r]);
        }
    };
    // window: Lambda and g of planes z-1, z, z+1; T and alpha2 of z and z+1
    double Lm[RW], gm[RW], tc[RW], ac[RW], Lc[RW], gc[RW], tp[RW], ap[RW], Lp[RW], gp[RW];
    load_plane(z0 - 1, tp, ap, Lm, gm);
    load_plane(z0, tc, ac, Lc, gc);
    double bound = 0.0;
    for (int z = z0; z < z1; ++z) {
        load_plane(z + 1, tp, ap, Lp, gp);
        const bool fB = a.perz ? nz > 1 : z > 0;
        const bool fF = a.perz ? nz > 1 : z < nz - 1;
        // the output rows' m1, m2 (1/C rebuilt) or 1/C, both rows at once
        double m1o[kRows3 + 1], m2o[kRows3 + 1], rco[kRows3 + 1];
#pragma unroll
        for (int r = 1; r <= kRows3; ++r) {
            const int y = y0 + r - 1;
            const unsigned o = out_lane && y < ny ? (unsigned)z * plane + (unsigned)y * (unsigned)nx + (unsigned)xg : 0u;
            m1o[r] = a.rebuild ? a.m1[o] : 0.0;
            m2o[r] = a.rebuild ? a.m2[o] : 0.0;
            rco[r] = a.rebuild ? 0.0 : a.rC_in[o];
        }
#pragma unroll
        for (int r = 1; r <= kRows3; ++r) {
            const int y = y0 + r - 1;
            const double L = Lc[r];
            const double Ll = from_left(L), Lr = from_right(L);
            const float Lf = (float)L;
            const float Llf = from_left(Lf), Lrf = from_right(Lf);
            const double gl = from_left(gc[r]), gr = from_right(gc[r]);
            if (out_lane && y < ny) {
                const unsigned o = (unsigned)z * plane + (unsigned)y * (unsigned)nx + (unsigned)xg;
                const bool fD = a.pery ? ny > 1 : y > 0;
                const bool fU = a.pery ? ny > 1 : y < ny - 1;
                if constexpr (kRelax) {
                    a.Tn_out[o] = tc[r];
                    a.a2_out[o] = ac[r];
                }
                double rc;
                if (a.rebuild) {
                    rc = inv_heat_capacity(a.ph, a.eps, tc[r], ac[r], m1o[r], m2o[r]);
                    a.rC[o] = rc;
                    if (a.rC32) a.rC32[o] = (float)rc;
                } else {
                    rc = rco[r];
                }
                if (a.Lam) a.Lam[o] = L;
                if (a.Lam32) a.Lam32[o] = Lf;
                // faces in the order -x, +x, -y, +y, -z, +z
                double d = 0.0;
                if (fL) d += a.wx * fmean<double>(L, Ll, a.face);
                if (fR) d += a.wx * fmean<double>(L, Lr, a.face);
                if (fD) d += a.wy * fmean<double>(L, Lc[r - 1], a.face);
                if (fU) d += a.wy * fmean<double>(L, Lc[r + 1], a.face);
                if (fB) d += a.wz * fmean<double>(L, Lm[r], a.face);
                if (fF) d += a.wz * fmean<double>(L, Lp[r], a.face);
                bound = fmax(bound, 2.0 * d * rc);
                if (q) {
                    const double La = (double)Lf, rf = (double)(float)rc, ga = gc[r];
                    double S = 0.0;
                    if (fL) S += a.wx * fmean<double>(La, (double)Llf, a.face) * (ga - gl);
                    if (fR) S += a.wx * fmean<double>(La, (double)Lrf, a.face) * (ga - gr);
                    if (fD) S += a.wy * fmean<double>(La, (double)(float)Lc[r - 1], a.face) * (ga - gc[r - 1]);
                    if (fU) S += a.wy * fmean<double>(La, (double)(float)Lc[r + 1], a.face) * (ga - gc[r + 1]);
                    if (fB) S += a.wz * fmean<double>(La, (double)(float)Lm[r], a.face) * (ga - gm[r]);
                    if (fF) S += a.wz * fmean<double>(La, (double)(float)Lp[r], a.face) * (ga - gp[r]);
                    a.q32[o] = (float)(-a.tau * rf * S);
                    if (a.w0) a.w0[o] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            Lm[r] = Lc[r];
            gm[r] = gc[r];
            tc[r] = tp[r];
            ac[r] = ap[r];
            Lc[r] = Lp[r];
            gc[r] = gp[r];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
    if (lane == 0) {
        const int sl = wid % kSlots;
        atomicMax((unsigned long long*)(a.lam + sl), (unsigned long long)__double_as_longlong(bound + 0.0));
    }
}

}  // namespace

bool coeffs2d_applies(const DevGrid& g) { return g.nz == 1 || g.N < ((int64_t)1 << 32); }

void launch_coeffs2d(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                     const double* T, const double* alpha2, const double* m1, const double* m2, const double* Tn,
                     int rebuild, double* Lam, double* rC, float* Lam32, float* rC32, float* q32, float* w0,
                     double* lam, const double* T2_relax, double* Tn_out, double* a2_out) {
    Coef2DArgs a{};
    a.ph = ph;
    a.T = T;
    a.T2 = T2_relax;
    a.Tn_out = Tn_out;
    a.a2_out = a2_out;
    a.alpha2 = alpha2;
    a.m1 = m1;
    a.m2 = m2;
    a.g = Tn;
    a.rC_in = rC;
    a.Lam = Lam;
    a.rC = rC;
    a.Lam32 = Lam32;
    a.rC32 = rC32;
    a.q32 = q32;
    a.w0 = w0;
    a.lam = lam;
    a.nx = g.nx;
    a.ny = g.ny;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.wx = g.w[0];
    a.wy = g.w[1];
    a.tau = tau;
    a.eps = eps;
    a.face = face;
    a.rebuild = rebuild;
    a.tiles_x = (g.nx + kOut - 1) / kOut;
    if (T2_relax) a.rebuild = 1;
    if (g.nz == 1) {
        a.strips = a.tiles_x * ((g.ny + kRows - 1) / kRows);
        const int blocks = (a.strips + kWaves - 1) / kWaves;
        if (ph.spitzer) {
            if (T2_relax) hipLaunchKernelGGL((k_coeffs2d<true, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
            else hipLaunchKernelGGL((k_coeffs2d<false, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
        } else {
            if (T2_relax) hipLaunchKernelGGL((k_coeffs2d<true, false>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
            else hipLaunchKernelGGL((k_coeffs2d<false, false>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
        }
        return;
    }
    a.nz = g.nz;
    a.perz = g.per[2];
    a.wz = g.w[2];
    a.tiles_y = (g.ny + kRows3 - 1) / kRows3;
    // z chunks sized for about 4096 waves, 4..64 planes each
    const int64_t cols = (int64_t)a.tiles_x * a.tiles_y;
    int64_t zc = (int64_t)g.nz * cols / 4096;
    zc = zc < 4 ? 4 : (zc > 64 ? 64 : zc);
    a.zc = (int)zc;
    a.strips = (int)(cols * ((g.nz + a.zc - 1) / a.zc));
    const int blocks = (a.strips + kWaves - 1) / kWaves;
    if (ph.spitzer) {
        if (T2_relax) hipLaunchKernelGGL((k_coeffs3d<true, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
        else hipLaunchKernelGGL((k_coeffs3d<false, true>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
    } else {
        if (T2_relax) hipLaunchKernelGGL((k_coeffs3d<true, false>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
        else hipLaunchKernelGGL((k_coeffs3d<false, false>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, s, a);
    }
}

}  // namespace tlim
