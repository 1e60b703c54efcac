// Inner LIM stages (eq. LIM) with temporal blocking for 2D grids.
//
// One stage of eq. LIM is a 5-point explicit update,
//   v^(m)_a = c_m (G_a + tau b_m v^(m-1)_a - sum_f kappa_af (v^(m-1)_a - v^(m-1)_f)),
//   kappa_af = tau / C_a * w_f * Lambda_f,
// with G = g = T^n + tau f (FP64 form) or G = -tau A' g (FP32 correction form,
// where v is the correction w = v - g).  The final stage (b = 0) of the FP64
// form is the same update with c = 1.
//
// k_tb2d advances K stages per launch.  A workgroup of NW wave64s
// loads a 64 x (NW*ROWS) extended tile once (v, G, Lambda, 1/C; one
// coalesced 64-wide row per wave per field), builds the four kappa of every
// cell in registers, and then runs the K stages out of registers:
//   - x-neighbours come from the adjacent lanes through DPP wave shifts;
//   - y-neighbours are the lane's own registers (each lane owns ROWS
//     consecutive cells of one column), except at the seams between waves,
//     which go through a double-buffered LDS row (one barrier per stage).
// Cells within K of the extended tile's edge go stale one ring per stage;
// the inner (64-2K) x (NW*ROWS-2K) cells are exact and written out.
// Grids of at least 128 rows use 16 waves (128-row tiles, one workgroup per
// CU, up to 10 stages per launch), smaller ones 8 waves (64-row tiles, up to
// 8 stages).  Every workgroup of a launch is resident at once on the 1024^2
// grids, so a launch costs one load phase plus its stages: the taller tile
// halves the halo per stage and lets a Picard pass of 15-20 stages run in
// two launches instead of three.
// Bytes per launch: 4 words read per extended cell + 1 word written per
// output cell, for K stages.
#include <hip/hip_runtime.h>

#include "tlim_device.h"
#include "tlim_sweep.h"

namespace tlim {

namespace {

using tb::ROWS;
using tb::row_index;
using tb::lane_value;

constexpr int KMAX_TB = 10;     // stages per launch, 16-wave tiles
constexpr int KMAX_SHORT = 8;   // stages per launch, 8-wave tiles
constexpr int TALL_ROWS = 128;  // grids with at least this many rows use 16-wave tiles
using tb::from_left;
using tb::from_right;
using tb::fmean;
using tb::fold;

template <typename R>
struct TBArgs {
    const R* v;
    const R* G;
    const R* Lam;
    const R* rC;
    R* out;
    const double* lam;       // accumulator row of lambda_max (NULL: use tb)
    const double* Tit;       // previous iterate: accumulate the pass reductions (last launch, FP64)
    PassSlots ps;
    R* stages;               // non-NULL: the result of stage s < K-1 also goes to stages + (s+1)*sstride
    int64_t sstride;
    // FP32 correction form: with g64 != NULL the launch's last stage is the
    // final one, evaluated in double from g64 + w with rC64, into out64
    const double* g64;
    const double* rC64;
    double* out64;
    double g64w[2];          // face weights in double for that stage
    // Launch with the final stage: with lam_next != NULL also the next
    // Picard pass's conductivities (Lam_next) and Gershgorin bound (max into
    // the row lam_next) from the new iterate; the output ring is then one
    // cell narrower (halo H = K + 1) so that the new iterate is known on the
    // neighbours of every output cell.
    double* lam_next;
    const double* alpha2;
    double* Lam_next;        // FP64
    float* Lam32_next;       // FP32 correction form: float conductivities and
    float* q32_next;         // the correction source -tau rC' D' g of the next pass
    // partial densities (rho = m1 + m2 of the Spitzer-Harm law, and the
    // relaxation); next_step: the next step's relaxation and first
    // coefficients instead of the next pass's (relaxed T and alpha2 to
    // Tn_next/a2_next; 1/C is unchanged with equal p_inf)
    const double* m1;
    const double* m2;
    int next_step;
    double* Tn_next;
    double* a2_next;
    double eps;
    DevPhases ph;
    int nx, ny, perx, pery;
    R wx, wy, tau;
    int K, H, face, tiles_x, ox, oy;
    double taud;
    double tb[KMAX_TB], chat[KMAX_TB];
};

// kSH: the conductivities built in the epilogue follow the Spitzer-Harm law
// in some phase (its logarithms would otherwise take registers from the
// power-law kernels).
template <typename R, int NW, bool kKeep, bool kSH>
__global__ void __launch_bounds__(64 * NW, 4) k_tb2d(TBArgs<R> a) {
    constexpr int WAVES = NW;
    constexpr int EXT_Y = NW * ROWS;
    __shared__ R sh_lo[2][WAVES][64];  // row 0 of each wave (the "up" row of the wave below)
    __shared__ R sh_hi[2][WAVES][64];  // row ROWS-1 of each wave (the "down" row of the wave above)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Lambda of a cell in the epilogues (rho = m1 + m2 used only under the
    // Spitzer-Harm law)
    auto law = [&](double t, double a2, double m1, double m2) -> double {
        if constexpr (kSH) return phys::cell_conductivity(a.ph, t, a2, m1 + m2);
        else return phys::cell_conductivity_pow(a.ph, t, a2);
    };
    const int K = a.K, H = a.H;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int xg = tx * a.ox - H + lane;
    const int yg0 = ty * a.oy - H + wv * ROWS;
    const int xi = fold(xg, a.nx, a.perx);
    const int yi0 = fold(yg0, a.ny, a.pery);
    const bool inx = xg >= 0 && xg < a.nx;
    const bool fL = a.perx ? a.nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? a.nx > 1 : (inx && xg < a.nx - 1);

    constexpr bool kFloat = sizeof(R) == 4;
    const bool fin = kFloat && a.g64 != nullptr;
    // In double the source G lives in LDS (read once per cell and stage):
    // the four kappa and v already take 80 of the 128 VGPRs that four
    // workgroups per CU leave, and G in registers spills.
    constexpr bool kGinLds = !kFloat;
    __shared__ R sG[kGinLds ? EXT_Y : 1][64];
    R v[ROWS], G[ROWS], kL[ROWS], kR[ROWS], kD[ROWS], kU[ROWS];
    const bool same = a.v == a.G;
    R Lk[ROWS];     // cell conductivities, kept for a fused FP64 final stage
    R Ldk = 0, Luk = 0;
    {
        R L[ROWS], t[ROWS];
        if constexpr (kFloat) {
            // every row's words in flight before the first is used (the
            // double kernels load row by row, as in the epilogue)
            int64_t idx[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) idx[r] = (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + xi;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                v[r] = a.v[idx[r]];
                L[r] = a.Lam[idx[r]];
                t[r] = a.rC[idx[r]];
            }
            // the first launch of a pass starts from v^(0) = T^n = g
            if (same) {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) G[r] = v[r];
            } else {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) G[r] = a.G[idx[r]];
            }
#pragma unroll
            for (int r = 0; r < ROWS; ++r) t[r] = a.tau * t[r];
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t idx = (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + xi;
                v[r] = a.v[idx];
                // the first launch of a pass starts from v^(0) = T^n = g
                sG[wv * ROWS + r][lane] = same ? v[r] : a.G[idx];
                L[r] = a.Lam[idx];
                t[r] = a.tau * a.rC[idx];
            }
        }
        sh_lo[0][wv][lane] = L[0];
        sh_hi[0][wv][lane] = L[ROWS - 1];
        __syncthreads();
        const R Ldn = wv > 0 ? sh_hi[0][wv - 1][lane] : L[0];
        const R Lup = wv < WAVES - 1 ? sh_lo[0][wv + 1][lane] : L[ROWS - 1];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = yg0 + r;
            const bool iny = y >= 0 && y < a.ny;
            const bool fD = a.pery ? a.ny > 1 : (iny && y > 0);
            const bool fU = a.pery ? a.ny > 1 : (iny && y < a.ny - 1);
            const R Ll = from_left(L[r]), Lr = from_right(L[r]);
            const R Ld = r > 0 ? L[r - 1] : Ldn;
            const R Lu = r < ROWS - 1 ? L[r + 1] : Lup;
            kL[r] = fL ? t[r] * a.wx * fmean<R>(L[r], Ll, a.face) : R(0);
            kR[r] = fR ? t[r] * a.wx * fmean<R>(L[r], Lr, a.face) : R(0);
            kD[r] = fD ? t[r] * a.wy * fmean<R>(L[r], Ld, a.face) : R(0);
            kU[r] = fU ? t[r] * a.wy * fmean<R>(L[r], Lu, a.face) : R(0);
        }
        if constexpr (kFloat) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) Lk[r] = L[r];
            Ldk = Ldn;
            Luk = Lup;
        }
    }
    // lambda_G of the pass from its accumulator row (every wave folds it)
    double lamv = 0.0;
    if (a.lam) {
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) lamv = fmax(lamv, a.lam[lane + 64 * k]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lamv = fmax(lamv, __shfl_xor(lamv, o, 64));
    }
    // Stage parameters: lane s holds tau*b_s and c_s = 1/(1 + tau*b_s) of
    // stage s; the stage loop reads them with readlane.
    double ptb = 0.0, pcm = 1.0;
    if (lane < K) {
        ptb = a.lam ? a.taud * lamv * a.chat[lane] : a.tb[lane];
        pcm = 1.0 / (1.0 + ptb);
    }
    // Stage s exchanges the seam rows through LDS buffer (s+1)&1; buffer 0
    // held the Lambda seams, whose reads all precede the first barrier below.
    // The end waves read a valid row and discard it (no branch).
    const int Kin = fin ? K - 1 : K;
    const int wdn = wv > 0 ? wv - 1 : 0, wup = wv < WAVES - 1 ? wv + 1 : wv;
    for (int s = 0; s < Kin; ++s) {
        const int buf = (s + 1) & 1;
        sh_lo[buf][wv][lane] = v[0];
        sh_hi[buf][wv][lane] = v[ROWS - 1];
        __syncthreads();
        const R sdn = sh_hi[buf][wdn][lane], sup = sh_lo[buf][wup][lane];
        const R vdn = wv > 0 ? sdn : v[0];
        const R vup = wv < WAVES - 1 ? sup : v[ROWS - 1];
        const double tbd = lane_value(ptb, s);
        const R cm = (R)lane_value(pcm, s), tb = (R)tbd;
        // Each face difference is formed once and shared by the face's two
        // cells: c - c_left is minus the left neighbour's c - c_right, and
        // c - c_below minus the row below's c - c_above (exact in floating
        // point, so S is the same number as with four differences per cell).
        R ddn = v[0] - vdn;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const R c = v[r];
            const R up = r < ROWS - 1 ? v[r + 1] : vup;
            const R drt = c - from_right(c);
            const R dlf = -from_left(drt);
            const R dup = c - up;
            const R S = kL[r] * dlf + kR[r] * drt + kD[r] * ddn + kU[r] * dup;
            R Gr;
            if constexpr (kGinLds) Gr = sG[wv * ROWS + r][lane];
            else Gr = G[r];
            v[r] = cm * (Gr + tb * c - S);
            ddn = -dup;
        }
        // the output cells are exact after every stage: keep the intermediate
        // stages when asked (the adjoint's recomputation)
        if (kKeep && s + 1 < K && lane >= H && lane < 64 - H && xg < a.nx) {
            R* dst = a.stages + (int64_t)(s + 1) * a.sstride;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int row = wv * ROWS + r;
                const int y = yg0 + r;
                if (row >= H && row < EXT_Y - H && y < a.ny) dst[(int64_t)y * a.nx + xg] = v[r];
            }
        }
    }
    // Final stage (b = 0) of the FP32 correction form, in double on v = g + w:
    // T = g - tau rC64 sum_f w_f mean(Lambda'_a, Lambda'_b) (v_a - v_b), with
    // Lambda' the float conductivities.  Sfin holds the flux sum, gfin g.
    double Sfin[ROWS], gfin[ROWS];
    if constexpr (kFloat) {
        if (fin) {
            __shared__ double dsh_lo[WAVES][64], dsh_hi[WAVES][64];
            double vf[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t idx = (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + xi;
                gfin[r] = a.g64[idx];
                vf[r] = gfin[r] + (double)v[r];
            }
            dsh_lo[wv][lane] = vf[0];
            dsh_hi[wv][lane] = vf[ROWS - 1];
            __syncthreads();
            const double vdn = wv > 0 ? dsh_hi[wv - 1][lane] : vf[0];
            const double vup = wv < WAVES - 1 ? dsh_lo[wv + 1][lane] : vf[ROWS - 1];
            const double wxd = a.g64w[0], wyd = a.g64w[1];
            double prev = vdn;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int y = yg0 + r;
                const bool iny = y >= 0 && y < a.ny;
                const bool fD = a.pery ? a.ny > 1 : (iny && y > 0);
                const bool fU = a.pery ? a.ny > 1 : (iny && y < a.ny - 1);
                const double c = vf[r];
                const double up = r < ROWS - 1 ? vf[r + 1] : vup;
                const double La = (double)Lk[r];
                const double Ll = (double)from_left(Lk[r]), Lr = (double)from_right(Lk[r]);
                const double Ld = (double)(r > 0 ? Lk[r - 1] : Ldk);
                const double Lu = (double)(r < ROWS - 1 ? Lk[r + 1] : Luk);
                const double lf = from_left(c), rt = from_right(c);
                double S = 0.0;
                if (fL) S += wxd * fmean<double>(La, Ll, a.face) * (c - lf);
                if (fR) S += wxd * fmean<double>(La, Lr, a.face) * (c - rt);
                if (fD) S += wyd * fmean<double>(La, Ld, a.face) * (c - prev);
                if (fU) S += wyd * fmean<double>(La, Lu, a.face) * (c - up);
                prev = c;
                Sfin[r] = S;
            }
            if (a.lam_next) {
                // Coefficients of the next Picard pass at the new iterate T
                // (valid K cells in from the edge; g = T^n): the conductivity
                // in double for the bound, its float rounding and the source
                // q = -tau rC' D' g from the float-rounded Lambda' and rC', at
                // the output cells (K+1 in), faces in the order -x, +x, -y, +y.
                double Ln[ROWS], rc[ROWS], a2v[ROWS], m1v[ROWS], m2v[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const int64_t idx = (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + xi;
                    rc[r] = a.rC64[idx];
                    a2v[r] = a.alpha2[idx];
                    m1v[r] = kSH ? a.m1[idx] : 0.0;
                    m2v[r] = kSH ? a.m2[idx] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const double tn = gfin[r] - a.taud * rc[r] * Sfin[r];
                    Ln[r] = law(tn, a2v[r], m1v[r], m2v[r]);
                }
                __shared__ double esh[4][WAVES][64];  // seams of Lambda and g
                esh[0][wv][lane] = Ln[0];
                esh[1][wv][lane] = Ln[ROWS - 1];
                esh[2][wv][lane] = gfin[0];
                esh[3][wv][lane] = gfin[ROWS - 1];
                __syncthreads();
                const double Ldn = wv > 0 ? esh[1][wv - 1][lane] : Ln[0];
                const double Lup = wv < WAVES - 1 ? esh[0][wv + 1][lane] : Ln[ROWS - 1];
                const double gdn = wv > 0 ? esh[3][wv - 1][lane] : gfin[0];
                const double gup = wv < WAVES - 1 ? esh[2][wv + 1][lane] : gfin[ROWS - 1];
                const double wxd = a.g64w[0], wyd = a.g64w[1];
                double bound = 0.0;
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const double L = Ln[r];
                    const double Ll = from_left(L), Lr = from_right(L);
                    const float Lf = (float)L;
                    const float Llf = from_left(Lf), Lrf = from_right(Lf);
                    const double gl = from_left(gfin[r]), gr = from_right(gfin[r]);
                    const double Ld = r > 0 ? Ln[r - 1] : Ldn, Lu = r < ROWS - 1 ? Ln[r + 1] : Lup;
                    const double gd = r > 0 ? gfin[r - 1] : gdn, gu = r < ROWS - 1 ? gfin[r + 1] : gup;
                    const int row = wv * ROWS + r;
                    const int y = yg0 + r;
                    if (lane >= H && lane < 64 - H && xg < a.nx && row >= H && row < EXT_Y - H && y < a.ny) {
                        const bool fD = a.pery ? a.ny > 1 : y > 0;
                        const bool fU = a.pery ? a.ny > 1 : y < a.ny - 1;
                        const int64_t o = (int64_t)y * a.nx + xg;
                        double d = 0.0;
                        if (fL) d += wxd * fmean<double>(L, Ll, a.face);
                        if (fR) d += wxd * fmean<double>(L, Lr, a.face);
                        if (fD) d += wyd * fmean<double>(L, Ld, a.face);
                        if (fU) d += wyd * fmean<double>(L, Lu, a.face);
                        bound = fmax(bound, 2.0 * d * rc[r]);
                        const double La = (double)Lf, rf = (double)(float)rc[r], ga = gfin[r];
                        double Sq = 0.0;
                        if (fL) Sq += wxd * fmean<double>(La, (double)Llf, a.face) * (ga - gl);
                        if (fR) Sq += wxd * fmean<double>(La, (double)Lrf, a.face) * (ga - gr);
                        if (fD) Sq += wyd * fmean<double>(La, (double)(float)Ld, a.face) * (ga - gd);
                        if (fU) Sq += wyd * fmean<double>(La, (double)(float)Lu, a.face) * (ga - gu);
                        a.Lam32_next[o] = Lf;
                        a.q32_next[o] = (float)(-a.taud * rf * Sq);
                    }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
                if (lane == 0) {
                    const int sl = (int)(((int64_t)blockIdx.x * WAVES + wv) % kSlots);
                    atomicMax((unsigned long long*)(a.lam_next + sl),
                              (unsigned long long)__double_as_longlong(bound + 0.0));
                }
            }
        }
    }
    double dmax = 0.0, tmax = 0.0, bad = 0.0;
    // the first pass's previous iterate is T^n = g, already on chip
    const bool tit_is_g = kFloat ? (fin && a.Tit == a.g64) : (const void*)a.Tit == (const void*)a.G;
    // Float kernels read the epilogue's words of every row up front, before
    // any is used (bit r of outm: row r of this lane is an output cell).  The
    // double kernels read them row by row: there the registers that batching
    // takes cost more than the load order gains (measured).
    unsigned outm = 0;
    if (lane >= H && lane < 64 - H && xg < a.nx) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int row = wv * ROWS + r;
            if (row >= H && row < EXT_Y - H && yg0 + r < a.ny) outm |= 1u << r;
        }
    }
    auto out_at = [&](int r) -> int64_t { return (outm >> r) & 1u ? (int64_t)(yg0 + r) * a.nx + xg : 0; };
    double titv[ROWS], rcf[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        titv[r] = 0.0;
        rcf[r] = 0.0;
    }
    if constexpr (kFloat) {
        if (a.Tit && !tit_is_g) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) titv[r] = a.Tit[out_at(r)];
        }
        if (fin) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) rcf[r] = a.rC64[out_at(r)];
        }
    }
    if (lane >= H && lane < 64 - H && xg < a.nx) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int row = wv * ROWS + r;
            if (row >= H && row < EXT_Y - H && yg0 + r < a.ny) {
                const int64_t o = (int64_t)(yg0 + r) * a.nx + xg;
                double tnew;
                if (fin) {
                    tnew = gfin[r] - a.taud * rcf[r] * Sfin[r];
                    a.out64[o] = tnew;
                } else {
                    a.out[o] = v[r];
                    tnew = (double)v[r];
                }
                if (a.Tit) {
                    const double tn = tnew;
                    double tit;
                    if (tit_is_g) {
                        if constexpr (kFloat) tit = gfin[r];
                        else tit = (double)sG[wv * ROWS + r][lane];
                    } else {
                        if constexpr (kFloat) tit = titv[r];
                        else tit = a.Tit[o];
                    }
                    dmax = fmax(dmax, fabs(tn - tit));
                    tmax = fmax(tmax, fabs(tn));
                    if (!(tn > 0.0) || isinf(tn)) bad += 1.0;
                }
            }
        }
    }
    if (a.Tit) {
        // wave-level fold, then lane 0 of every wave adds to a slot of the rows
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
            tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
            bad += __shfl_xor(bad, o, 64);
        }
        if (lane == 0) {
            const int sl = (int)(((int64_t)blockIdx.x * WAVES + wv) % kSlots);
            atomicMax((unsigned long long*)(a.ps.dmax + sl), (unsigned long long)__double_as_longlong(dmax + 0.0));
            atomicMax((unsigned long long*)(a.ps.tmax + sl), (unsigned long long)__double_as_longlong(tmax + 0.0));
            if (bad != 0.0) atomicAdd(a.ps.bad + sl, bad);
        }
    }
    if constexpr (!kFloat) {
        if (a.lam_next) {
            // Coefficients of the next Picard pass at the new iterate v (valid
            // K cells in from the edge): Lambda = sum_k alpha_k lambda_k(v),
            // and at the output cells (K+1 in) the bound 2 rC sum_f w_f
            // mean(Lambda_a, Lambda_b), faces in the order -x, +x, -y, +y.
            // With m1 the next step's instead: every cell relaxed from
            // (alpha2, v, v, m1, m2) first, Lambda and 1/C at the relaxed state.
            const bool next_step = a.next_step != 0;
            double Ln[ROWS], Tr[ROWS], ar[ROWS], rr[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t idx = (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + xi;
                const double a2v = a.alpha2[idx];
                if (next_step) {
                    const double m1 = a.m1[idx], m2 = a.m2[idx];
                    phys::relax_cell(a.ph, a.eps, a2v, v[r], v[r], m1, m2, Tr[r], ar[r]);
                    rr[r] = phys::inv_heat_capacity(a.ph, a.eps, Tr[r], ar[r], m1, m2);
                    Ln[r] = law(Tr[r], ar[r], m1, m2);
                } else if constexpr (kSH) {
                    Ln[r] = law(v[r], a2v, a.m1[idx], a.m2[idx]);
                } else {
                    Ln[r] = law(v[r], a2v, 0.0, 0.0);
                }
            }
            // the seam buffer not used by the last stage: its reads all
            // precede that stage's barrier
            const int b2 = (K + 1) & 1;
            sh_lo[b2][wv][lane] = Ln[0];
            sh_hi[b2][wv][lane] = Ln[ROWS - 1];
            __syncthreads();
            const double Ldn = wv > 0 ? sh_hi[b2][wv - 1][lane] : Ln[0];
            const double Lup = wv < WAVES - 1 ? sh_lo[b2][wv + 1][lane] : Ln[ROWS - 1];
            double bound = 0.0;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const double Ll = from_left(Ln[r]), Lr = from_right(Ln[r]);
                const double Ld = r > 0 ? Ln[r - 1] : Ldn;
                const double Lu = r < ROWS - 1 ? Ln[r + 1] : Lup;
                const int row = wv * ROWS + r;
                const int y = yg0 + r;
                if (lane >= H && lane < 64 - H && xg < a.nx && row >= H && row < EXT_Y - H && y < a.ny) {
                    const bool fD = a.pery ? a.ny > 1 : y > 0;
                    const bool fU = a.pery ? a.ny > 1 : y < a.ny - 1;
                    const int64_t o = (int64_t)y * a.nx + xg;
                    double d = 0.0;
                    if (fL) d += a.wx * fmean<double>(Ln[r], Ll, a.face);
                    if (fR) d += a.wx * fmean<double>(Ln[r], Lr, a.face);
                    if (fD) d += a.wy * fmean<double>(Ln[r], Ld, a.face);
                    if (fU) d += a.wy * fmean<double>(Ln[r], Lu, a.face);
                    const double rc = next_step ? rr[r] : a.rC[o];
                    bound = fmax(bound, 2.0 * d * rc);
                    a.Lam_next[o] = Ln[r];
                    if (next_step) {
                        a.Tn_next[o] = Tr[r];
                        a.a2_next[o] = ar[r];
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
            if (lane == 0) {
                const int sl = (int)(((int64_t)blockIdx.x * WAVES + wv) % kSlots);
                atomicMax((unsigned long long*)(a.lam_next + sl), (unsigned long long)__double_as_longlong(bound + 0.0));
            }
        }
    }
}

template <typename R>
int launch_tb2d(hipStream_t s, const DevGrid& g, int face, const R* v, const R* G, const R* Lam, const R* rC,
                R* out, Stages st, int count, double tau, const double* Tit, PassSlots ps, R* stages = nullptr,
                int64_t sstride = 0, const double* g64 = nullptr, const double* rC64 = nullptr,
                double* out64 = nullptr, const NextCoef* nc = nullptr) {
    TBArgs<R> a{};
    if (nc) {
        a.lam_next = nc->lam;
        a.alpha2 = nc->alpha2;
        a.Lam_next = nc->Lam;
        a.Lam32_next = nc->Lam32;
        a.q32_next = nc->q32;
        a.ph = nc->ph;
        a.m1 = nc->m1;
        a.m2 = nc->m2;
        a.next_step = nc->next_step;
        a.Tn_next = nc->Tn;
        a.a2_next = nc->a2;
        a.eps = nc->eps;
    }
    a.g64 = g64;
    a.rC64 = rC64;
    a.out64 = out64;
    a.g64w[0] = g.w[0];
    a.g64w[1] = g.w[1];
    a.stages = stages;
    a.sstride = sstride;
    const bool tall = g.ny >= TALL_ROWS;
    const int kmax = tall ? KMAX_TB : KMAX_SHORT;
    const int EXT_Y = (tall ? 16 : 8) * ROWS;
    int K = count < kmax ? count : kmax;
    a.v = v;
    a.G = G;
    a.Lam = Lam;
    a.rC = rC;
    a.out = out;
    a.lam = st.lam;
    a.Tit = Tit;
    a.ps = ps;
    a.nx = g.nx;
    a.ny = g.ny;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.wx = (R)g.w[0];
    a.wy = (R)g.w[1];
    a.tau = (R)tau;
    a.taud = tau;
    a.K = K;
    a.H = nc ? K + 1 : K;
    a.face = face;
    a.ox = 64 - 2 * a.H;
    a.oy = EXT_Y - 2 * a.H;
    a.tiles_x = (g.nx + a.ox - 1) / a.ox;
    int tiles_y = (g.ny + a.oy - 1) / a.oy;
    for (int k = 0; k < K; ++k) {
        if (st.lam) a.chat[k] = st.chat[k];
        else a.tb[k] = st.tb[k];
    }
    const dim3 grid((unsigned)(a.tiles_x * tiles_y));
    const bool sh = nc && nc->ph.spitzer;
    if (stages) {  // (no epilogue: the kept-stage launches of the adjoint's recompute)
        if (tall) hipLaunchKernelGGL((k_tb2d<R, 16, true, false>), grid, dim3(64 * 16), 0, s, a);
        else hipLaunchKernelGGL((k_tb2d<R, 8, true, false>), grid, dim3(64 * 8), 0, s, a);
    } else if (sh) {
        if (tall) hipLaunchKernelGGL((k_tb2d<R, 16, false, true>), grid, dim3(64 * 16), 0, s, a);
        else hipLaunchKernelGGL((k_tb2d<R, 8, false, true>), grid, dim3(64 * 8), 0, s, a);
    } else {
        if (tall) hipLaunchKernelGGL((k_tb2d<R, 16, false, false>), grid, dim3(64 * 16), 0, s, a);
        else hipLaunchKernelGGL((k_tb2d<R, 8, false, false>), grid, dim3(64 * 8), 0, s, a);
    }
    return K;
}

bool use_tb2d(const DevGrid& g, int count) {
    return g.nz == 1 && g.ny >= 8 * ROWS / 2 && count >= 2;
}

StageParam one_stage(const Stages& st) {
    StageParam sp;
    sp.lam = st.lam;
    sp.tb = st.lam ? 0.0 : st.tb[0];
    sp.chat = st.lam ? st.chat[0] : 0.0;
    return sp;
}

}  // namespace

int launch_sweeps64_keep(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                         const double* Lam, const double* rC, double* out, Stages st, int count, double tau,
                         double* stages, int64_t sstride) {
    if (use_tb2d(g, count))
        return launch_tb2d<double>(s, g, face, v, rhs, Lam, rC, out, st, count, tau, nullptr, PassSlots{}, stages,
                                   sstride);
    return -1;
}

int sweeps_per_launch(const DevGrid& g, int count) {
    if (!use_tb2d(g, count)) return 1;
    // as few launches as the tile allows, with equal stage counts: a launch
    // of K stages recomputes a ring of width K, so even launches waste least
    const int kmax = g.ny >= TALL_ROWS ? KMAX_TB : KMAX_SHORT;
    const int launches = (count + kmax - 1) / kmax;
    return (count + launches - 1) / launches;
}

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, Stages st, int count, bool last, double tau,
                    const double* Tit, PassSlots ps, const NextCoef* nc, bool* nc_done) {
    if (nc_done) *nc_done = false;
    if (use_tb2d(g, count)) {
        const bool with_nc = last && nc != nullptr;
        if (nc_done) *nc_done = with_nc;
        return launch_tb2d<double>(s, g, face, v, rhs, Lam, rC, out, st, count, tau, last ? Tit : nullptr, ps,
                                   nullptr, 0, nullptr, nullptr, nullptr, with_nc ? nc : nullptr);
    }
    if (use_z3d(g)) {
        if (last) launch_z3d<double>(s, g, face, v, rhs, Lam, rC, out, StageParam{nullptr, 0.0, 0.0}, tau, Tit, ps);
        else launch_z3d<double>(s, g, face, v, rhs, Lam, rC, out, one_stage(st), tau, nullptr, PassSlots{});
        return 1;
    }
    if (last) {
        // the final stage, b = 0, in flux form
        launch_final64(s, g, face, v, rhs, Lam, rC, out, tau, Tit, ps);
    } else {
        launch_stage64(s, g, face, v, rhs, Lam, rC, out, one_stage(st), tau);
    }
    return 1;
}

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* qn,
                    const float* Lam32, const float* rC32, float* out, Stages st, int count, bool last, double tau,
                    const double* rhs, const double* rC, double* out64, const double* Tit, PassSlots ps,
                    const NextCoef* nc, bool* nc_done) {
    if (nc_done) *nc_done = false;
    if (use_tb2d(g, count)) {
        if (last) {
            if (nc_done) *nc_done = nc != nullptr;
            return launch_tb2d<float>(s, g, face, w, qn, Lam32, rC32, nullptr, st, count, tau, Tit, ps, nullptr, 0,
                                      rhs, rC, out64, nc);
        }
        return launch_tb2d<float>(s, g, face, w, qn, Lam32, rC32, out, st, count, tau, nullptr, PassSlots{});
    }
    if (last) {
        if (use_z3d(g)) launch_z3d_final32(s, g, face, w, rhs, Lam32, rC, out64, tau, Tit, ps);
        else launch_final32(s, g, face, w, rhs, Lam32, rC, out64, tau, Tit, ps);
    } else if (use_z3d(g)) {
        launch_z3d<float>(s, g, face, w, qn, Lam32, rC32, out, one_stage(st), tau, nullptr, PassSlots{});
    } else {
        launch_stage32(s, g, face, w, qn, Lam32, rC32, out, one_stage(st), tau);
    }
    return 1;
}

}  // namespace tlim
