// Temporally blocked reverse stages of the LIM adjoint (2D grids, arithmetic
// face means).
//
// One stage of eq. LIM, v^(m) = c_m (g + tau b_m v^(m-1) - tau A v^(m-1)),
// A = C^-1 D with D symmetric, has the adjoint
//   lambda^(m-1) = c_m (tau b_m lambda^(m) - tau D C^-1 lambda^(m)).
// With psi = C^-1 lambda this is psi^(m-1) = c_m (tau b_m psi^(m) - tau A psi^(m)):
// the forward stage operator without source, so it runs on the same kappa
// = tau/C w Lambda_f and the same register-tiled scheme as the forward
// stages (tlim_sweep.hip).  Along the way the kernel accumulates
//   dgpsi += c_m psi^(m)                          (dL/dg = C dgpsi)
//   gLam  += c_m tau w/2 sum_f (v_b - v_a)^(m-1) (psi_a - psi_b)^(m)
// where dL/dLambda_f = c_m tau w (v_b - v_a)(psi_a - psi_b) and the arithmetic
// face mean gives dLambda_f/dLambda_a = 1/2.  The forward iterate v^(m-1) of
// every stage is read from the stored stages (one field per stage), one
// stage ahead of its use.
//
// The launch that reaches v^(0) can also finish the pass at its output
// cells (AdjCell): dL/dT^n += C (dgpsi + psi^(0)), the chain through the
// conductivity of the lagged iterate mu = gLam dLambda/dT(T^(it)) (added to
// dL/dT^n too for the first pass, whose iterate is T^n), and the two dL/dk0
// sums of the pass.
#include <hip/hip_runtime.h>

#include "tlim_device.h"
#include "tlim_sweep.h"

namespace tlim {

namespace {

using phys::powlaw;
using tb::EXT_Y;
using tb::fmean;
using tb::fold;
using tb::from_left;
using tb::from_right;
using tb::KMAX;
using tb::ROWS;
using tb::WAVES;

struct AdjArgs {
    const double* psi_in;
    const double* Lam;
    const double* rC;
    const double* stages;
    const double* v0;
    double* psi_out;
    double* dgpsi;
    double* gLam;
    int64_t sstride;
    int first, accumulate, mt;
    int nx, ny, perx, pery;
    double wx, wy, tau;
    int K, tiles_x, ox, oy;
    double cm[KMAX], tb[KMAX];
    AdjCell cell;  // cell.acc != NULL: finish the pass (this launch reaches v^(0))
};

// kSH: some phase follows the Spitzer-Harm law (the pass epilogue's
// conductivity derivatives take logarithms; the power-law kernel is kept
// free of them).
template <bool kSH>
__global__ void __launch_bounds__(64 * WAVES, 2) k_tb2d_adj(AdjArgs a) {
    __shared__ double sh_lo[2][WAVES][64];
    __shared__ double sh_hi[2][WAVES][64];
    __shared__ double sv_lo[2][WAVES][64];
    __shared__ double sv_hi[2][WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int K = a.K;
    const int tile = tb::xcd_block();  // tiles in XCD order (neighbours share an L2)
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int xg = tx * a.ox - K + lane;
    const int yg0 = ty * a.oy - K + wv * ROWS;
    const int xi = fold(xg, a.nx, a.perx);
    const bool inx = xg >= 0 && xg < a.nx;
    const bool fL = a.perx ? a.nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? a.nx > 1 : (inx && xg < a.nx - 1);
    const double hx = 0.5 * a.tau * a.wx, hy = 0.5 * a.tau * a.wy;

    int64_t idx[ROWS];
    double psi[ROWS], kL[ROWS], kR[ROWS], kD[ROWS], kU[ROWS], dga[ROWS], gla[ROWS];
    bool fD[ROWS], fU[ROWS];
    {
        double L[ROWS], t[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = yg0 + r;
            idx[r] = (int64_t)fold(y, a.ny, a.pery) * a.nx + xi;
            const double rc = a.rC[idx[r]];
            psi[r] = a.first ? a.psi_in[idx[r]] * rc : a.psi_in[idx[r]];
            L[r] = a.Lam[idx[r]];
            t[r] = a.tau * rc;
            dga[r] = a.accumulate ? a.dgpsi[idx[r]] : 0.0;
            gla[r] = a.accumulate ? a.gLam[idx[r]] : 0.0;
            const bool iny = y >= 0 && y < a.ny;
            fD[r] = a.pery ? a.ny > 1 : (iny && y > 0);
            fU[r] = a.pery ? a.ny > 1 : (iny && y < a.ny - 1);
        }
        sh_lo[0][wv][lane] = L[0];
        sh_hi[0][wv][lane] = L[ROWS - 1];
        __syncthreads();
        const double Ldn = wv > 0 ? sh_hi[0][wv - 1][lane] : L[0];
        const double Lup = wv < WAVES - 1 ? sh_lo[0][wv + 1][lane] : L[ROWS - 1];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const double Ll = from_left(L[r]), Lr = from_right(L[r]);
            const double Ld = r > 0 ? L[r - 1] : Ldn;
            const double Lu = r < ROWS - 1 ? L[r + 1] : Lup;
            kL[r] = fL ? t[r] * a.wx * fmean<double>(L[r], Ll, 0) : 0.0;
            kR[r] = fR ? t[r] * a.wx * fmean<double>(L[r], Lr, 0) : 0.0;
            kD[r] = fD[r] ? t[r] * a.wy * fmean<double>(L[r], Ld, 0) : 0.0;
            kU[r] = fU[r] ? t[r] * a.wy * fmean<double>(L[r], Lu, 0) : 0.0;
        }
    }
    const double gxl = fL ? hx : 0.0, gxr = fR ? hx : 0.0;
    // forward iterate v^(m-1) of stage m = mt - s, loaded one stage ahead
    auto vsrc = [&](int s) { const int j = a.mt - 1 - s; return j == 0 ? a.v0 : a.stages + (int64_t)j * a.sstride; };
    double vnext[ROWS];
    {
        const double* p = vsrc(0);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) vnext[r] = p[idx[r]];
    }
    for (int s = 0; s < K; ++s) {
        const int buf = (s + 1) & 1;
        double v[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) v[r] = vnext[r];
        if (s + 1 < K) {
            const double* p = vsrc(s + 1);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) vnext[r] = p[idx[r]];
        }
        sh_lo[buf][wv][lane] = psi[0];
        sh_hi[buf][wv][lane] = psi[ROWS - 1];
        sv_lo[buf][wv][lane] = v[0];
        sv_hi[buf][wv][lane] = v[ROWS - 1];
        __syncthreads();
        const double pdn = wv > 0 ? sh_hi[buf][wv - 1][lane] : psi[0];
        const double pup = wv < WAVES - 1 ? sh_lo[buf][wv + 1][lane] : psi[ROWS - 1];
        const double vdn = wv > 0 ? sv_hi[buf][wv - 1][lane] : v[0];
        const double vup = wv < WAVES - 1 ? sv_lo[buf][wv + 1][lane] : v[ROWS - 1];
        const double cm = a.cm[s], tb = a.tb[s];
        double prev = pdn;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const double c = psi[r];
            const double up = r < ROWS - 1 ? psi[r + 1] : pup;
            const double dLf = c - from_left(c), dRt = c - from_right(c), dDn = c - prev, dUp = c - up;
            const double va = v[r];
            const double eLf = from_left(va) - va, eRt = from_right(va) - va;
            const double eDn = (r > 0 ? v[r - 1] : vdn) - va;
            const double eUp = (r < ROWS - 1 ? v[r + 1] : vup) - va;
            const double G = gxl * eLf * dLf + gxr * eRt * dRt + (fD[r] ? hy : 0.0) * eDn * dDn +
                             (fU[r] ? hy : 0.0) * eUp * dUp;
            gla[r] += cm * G;
            dga[r] += cm * c;
            const double S = kL[r] * dLf + kR[r] * dRt + kD[r] * dDn + kU[r] * dUp;
            psi[r] = cm * (tb * c - S);
            prev = c;
        }
    }
    const AdjCell& cl = a.cell;
    double s0 = 0.0, s1 = 0.0;
    if (lane >= K && lane < 64 - K && xg < a.nx) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int row = wv * ROWS + r;
            const int y = yg0 + r;
            if (row >= K && row < EXT_Y - K && y < a.ny) {
                const int64_t o = (int64_t)y * a.nx + xg;
                if (cl.acc) {
                    const DevPhases& ph = cl.ph;
                    const double t = cl.Tit[o], a2 = cl.alpha2[o], gl = gla[r];
                    const double acc0 = cl.init ? 0.0 : cl.acc[o];
                    double acc_a = acc0 + (dga[r] + psi[r]) / a.rC[o];
                    double dL;
                    if constexpr (kSH) {
                        double dk[2];
                        phys::cell_conductivity_grad(ph, t, a2, cl.m1[o] + cl.m2[o], dk, dL);
                        s0 += gl * dk[0];
                        s1 += gl * dk[1];
                    } else {
                        const double a1 = 1.0 - a2;
                        const double x0 = t * ph.invT0[0], x1 = t * ph.invT0[1];
                        s0 += gl * a1 * powlaw(x0, ph.npow[0]);
                        s1 += gl * a2 * powlaw(x1, ph.npow[1]);
                        dL = 0.0;
                        if (ph.npow[0] != 0.0)
                            dL += a1 * ph.k0[0] * ph.npow[0] * powlaw(x0, ph.npow[0] - 1.0) * ph.invT0[0];
                        if (ph.npow[1] != 0.0)
                            dL += a2 * ph.k0[1] * ph.npow[1] * powlaw(x1, ph.npow[1] - 1.0) * ph.invT0[1];
                    }
                    const double mu = gl * dL;
                    cl.mu[o] = mu;
                    cl.acc[o] = cl.first_pass ? acc_a + mu : acc_a;
                } else {
                    a.psi_out[o] = psi[r];
                    a.dgpsi[o] = dga[r];
                    a.gLam[o] = gla[r];
                }
            }
        }
    }
    if (cl.acc) {
        // wave sums, then one atomic per wave into a slot of each row
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o, 64);
            s1 += __shfl_xor(s1, o, 64);
        }
        if (lane == 0) {
            const int sl = (int)(((int64_t)blockIdx.x * WAVES + wv) % kSlots);
            atomicAdd(cl.k0a + sl, s0);
            atomicAdd(cl.k0b + sl, s1);
        }
    }
}

}  // namespace

int launch_adjoint_sweeps(hipStream_t s, const DevGrid& g, int face, const double* psi_in, int first,
                          const double* Lam, const double* rC, const double* stages, const double* v0,
                          int64_t sstride, int mt,
                          double* psi_out, double* dgpsi, double* gLam, int accumulate, const double* cm,
                          const double* tb, int count, double tau, const AdjCell* cell) {
    if (!(g.nz == 1 && g.ny >= EXT_Y / 2 && face == 0)) return -1;
    AdjArgs a{};
    const int K = count < KMAX ? count : KMAX;
    if (cell && mt - K == 0) a.cell = *cell;
    a.psi_in = psi_in;
    a.Lam = Lam;
    a.rC = rC;
    a.stages = stages;
    a.v0 = v0;
    a.psi_out = psi_out;
    a.dgpsi = dgpsi;
    a.gLam = gLam;
    a.sstride = sstride;
    a.first = first;
    a.accumulate = accumulate;
    a.mt = mt;
    a.nx = g.nx;
    a.ny = g.ny;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.wx = g.w[0];
    a.wy = g.w[1];
    a.tau = tau;
    a.K = K;
    a.ox = 64 - 2 * K;
    a.oy = EXT_Y - 2 * K;
    a.tiles_x = (g.nx + a.ox - 1) / a.ox;
    const int tiles_y = (g.ny + a.oy - 1) / a.oy;
    for (int k = 0; k < K; ++k) {
        a.cm[k] = cm[k];
        a.tb[k] = tb[k];
    }
    if (a.cell.acc && a.cell.ph.spitzer)
        hipLaunchKernelGGL(k_tb2d_adj<true>, dim3((unsigned)(a.tiles_x * tiles_y)), dim3(64 * WAVES), 0, s, a);
    else
        hipLaunchKernelGGL(k_tb2d_adj<false>, dim3((unsigned)(a.tiles_x * tiles_y)), dim3(64 * WAVES), 0, s, a);
    return K;
}

}  // namespace tlim
