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
// loads an extended tile once (v, G, Lambda, 1/C; coalesced rows, one per
// wave and field), builds the four kappa of every cell in registers, and
// then runs the K stages out of registers:
//   - each lane owns C adjacent cells of a row (C = 1 or 2): x-neighbours
//     come from the lane's own cells or from the adjacent lanes through DPP
//     wave shifts;
//   - y-neighbours are the lane's own registers (each lane owns 8/C
//     consecutive rows), except at the seams between waves, which go
//     through a double-buffered LDS row (one barrier per stage).
// Cells within K of the extended tile's edge go stale one ring per stage;
// the inner (64C-2K) x (NW*8/C-2K) cells are exact and written out.
// Grids of at least 128 rows use 16 waves (64 x 128 tiles, or for the float
// stages on grids of at least 128 columns 128 x 64 tiles with two cells per
// lane), smaller ones 8 waves (64 x 64, up to 8 stages); one workgroup per
// CU, up to 10 stages per launch.  Every workgroup of a launch is resident at
// once on the 1024^2 grids, so a launch costs one load phase plus its stages:
// the 16-wave tiles halve the halo per stage against 64 x 64 and let a Picard
// pass of 15-20 stages run in two launches instead of three.  A 64-wide row
// of floats spans 3 cache lines for 2 lines of data (the rows start where
// the tile falls), a 128-wide one 5 for 4, and the lane's two cells come in
// one load: the FP32 form's launches that reach the final stage take 10%
// less time on the 128 x 64 tiles.  The double kernels gain nothing from
// them (5 lines for 4 against 9 for 8; the launch that relaxes and builds the
// next step's start runs slower), so they keep the 64 x 128 tiles.
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
constexpr int WIDE_COLS = 128;  // ... and 128-wide ones (two cells per lane) with at least this many columns
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
    int K, H, hx, face, tiles_x, ox, oy;
    int vzero;  // float stages: v is the all-zero start w0 = 0 (not read)
    double taud;
    double tb[KMAX_TB], chat[KMAX_TB];
};

// kSH: the conductivities built in the epilogue follow the Spitzer-Harm law
// in some phase (its logarithms would otherwise take registers from the
// power-law kernels).  C: cells per lane along x (1: 64-wide tiles of 8 rows
// per wave; 2: 128-wide tiles of 4 rows per wave, lane l owning cells 2l and
// 2l + 1, so that one of each cell's x-neighbours is in the lane itself).
template <typename R, int NW, int C, bool kKeep, bool kSH>
__global__ void __launch_bounds__(64 * NW, 4) k_tb2d(TBArgs<R> a) {
    constexpr int WAVES = NW;
    constexpr int RW = ROWS / C;       // rows per wave
    constexpr int EXT_X = 64 * C;
    constexpr int EXT_Y = NW * RW;
    __shared__ R sh_lo[2][WAVES][C][64];  // row 0 of each wave (the "up" row of the wave below)
    __shared__ R sh_hi[2][WAVES][C][64];  // row RW-1 of each wave (the "down" row of the wave above)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Lambda of a cell in the epilogues (rho = m1 + m2 used only under the
    // Spitzer-Harm law)
    auto law = [&](double t, double a2, double m1, double m2) -> double {
        if constexpr (kSH) return phys::cell_conductivity(a.ph, t, a2, m1 + m2);
        else return phys::cell_conductivity_pow(a.ph, t, a2);
    };
    // x-neighbours of cell j of this lane, from the lane's own cells or the
    // adjacent lanes (j is a compile-time index in the unrolled loops)
    auto left_of = [&](const auto (&x)[C], int j) { return j > 0 ? x[j - 1] : from_left(x[C - 1]); };
    auto right_of = [&](const auto (&x)[C], int j) { return j < C - 1 ? x[j + 1] : from_right(x[0]); };
    const int K = a.K, H = a.H;
    // the x ring: H, or with two cells per lane H rounded up to even, so that
    // the tile starts at an even column and a lane's two cells are adjacent
    // in memory (periodic x with an even width, or clamped walls)
    const int HX = a.hx;
    // tiles in XCD order: x-neighbours, whose extended tiles overlap by 2H
    // columns, mostly share an L2
    const int tile = tb::xcd_block();
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int yg0 = ty * a.oy - H + wv * RW;
    const int yi0 = fold(yg0, a.ny, a.pery);
    int xg[C], xi[C];
    bool fL[C], fR[C];
    // output column: cell j of this lane is at least HX in from the tile's x edges
    bool xo[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int xl = C * lane + j;
        xg[j] = tx * a.ox - HX + xl;
        xi[j] = fold(xg[j], a.nx, a.perx);
        const bool inx = xg[j] >= 0 && xg[j] < a.nx;
        fL[j] = a.perx ? a.nx > 1 : (inx && xg[j] > 0);
        fR[j] = a.perx ? a.nx > 1 : (inx && xg[j] < a.nx - 1);
        xo[j] = xl >= HX && xl < EXT_X - HX && xg[j] < a.nx;
    }
    // Two cells per lane come in one load of two words at column sx: the
    // pair (xi0, xi0 + 1) away from the walls, the clamped copies (both the
    // wall cell) beyond them; sel_j tells which word is cell j.
    const int sx = C == 2 ? min(xi[0], a.nx - 2) : xi[0];
    bool sel[C];
#pragma unroll
    for (int j = 0; j < C; ++j) sel[j] = xi[j] == sx;
    // first word of row r of the tile's lane (formed once per row: every
    // field's load of the row shares it)
    auto row_at = [&](int r) -> int64_t { return (int64_t)row_index(yi0, yg0, r, a.ny, a.pery) * a.nx + sx; };
    auto ld = [&](const auto* f, int64_t o, auto (&out)[C]) {
        if constexpr (C == 1) {
            out[0] = f[o];
        } else {
            using T = std::remove_cv_t<std::remove_reference_t<decltype(f[0])>>;
            struct alignas(sizeof(T)) Pair { T x, y; } pr;
            __builtin_memcpy(&pr, f + o, sizeof(Pair));
#pragma unroll
            for (int j = 0; j < C; ++j) out[j] = sel[j] ? pr.x : pr.y;
        }
    };
    auto yout = [&](int r) { const int row = wv * RW + r; return row >= H && row < EXT_Y - H && yg0 + r < a.ny; };

    constexpr bool kFloat = sizeof(R) == 4;
    const bool fin = kFloat && a.g64 != nullptr;
    // A float pass's first launch starts from w0 = 0, where its first stage
    // gives c_0 G exactly: v is then not read, and that stage is c_0 G.
    const bool vz = kFloat && !kKeep && a.vzero && a.v != a.G && (fin ? K - 1 : K) >= 1;
    // In double the source G lives in LDS (read once per cell and stage):
    // the four kappa and v already take 80 of the 128 VGPRs that four
    // workgroups per CU leave, and G in registers spills.
    constexpr bool kGinLds = !kFloat;
    __shared__ R sG[kGinLds ? EXT_Y : 1][C][64];
    R v[RW][C], G[RW][C], kL[RW][C], kR[RW][C], kD[RW][C], kU[RW][C];
    const bool same = a.v == a.G;
    R Lk[RW][C];     // cell conductivities, kept for a fused FP64 final stage
    R Ldk[C], Luk[C];
    {
        R L[RW][C], t[RW][C];
        if constexpr (kFloat) {
            // every row's words in flight before the first is used (the
            // double kernels load row by row, as in the epilogue)
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int64_t o = row_at(r);
                if (vz) {
#pragma unroll
                    for (int j = 0; j < C; ++j) v[r][j] = R(0);
                } else {
                    ld(a.v, o, v[r]);
                }
                ld(a.Lam, o, L[r]);
                ld(a.rC, o, t[r]);
            }
            // the first launch of a pass starts from v^(0) = T^n = g
            if (same) {
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < C; ++j) G[r][j] = v[r][j];
            } else {
#pragma unroll
                for (int r = 0; r < RW; ++r) ld(a.G, row_at(r), G[r]);
            }
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) t[r][j] = a.tau * t[r][j];
        } else {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int64_t o = row_at(r);
                // the first launch of a pass starts from v^(0) = T^n = g (G
                // is then not read)
                if constexpr (C == 1) {
                    v[r][0] = a.v[o];
                    sG[wv * RW + r][0][lane] = same ? v[r][0] : a.G[o];
                    L[r][0] = a.Lam[o];
                    t[r][0] = a.tau * a.rC[o];
                    continue;
                }
                R Gr[C];
                ld(a.v, o, v[r]);
                if (same) {
#pragma unroll
                    for (int j = 0; j < C; ++j) Gr[j] = v[r][j];
                } else {
                    ld(a.G, o, Gr);
                }
                ld(a.Lam, o, L[r]);
                ld(a.rC, o, t[r]);
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    sG[wv * RW + r][j][lane] = Gr[j];
                    t[r][j] = a.tau * t[r][j];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
            sh_lo[0][wv][j][lane] = L[0][j];
            sh_hi[0][wv][j][lane] = L[RW - 1][j];
        }
        __syncthreads();
        R Ldn[C], Lup[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            Ldn[j] = wv > 0 ? sh_hi[0][wv - 1][j][lane] : L[0][j];
            Lup[j] = wv < WAVES - 1 ? sh_lo[0][wv + 1][j][lane] : L[RW - 1][j];
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int y = yg0 + r;
            const bool iny = y >= 0 && y < a.ny;
            const bool fD = a.pery ? a.ny > 1 : (iny && y > 0);
            const bool fU = a.pery ? a.ny > 1 : (iny && y < a.ny - 1);
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const R Ll = left_of(L[r], j), Lr = right_of(L[r], j);
                const R Ld = r > 0 ? L[r - 1][j] : Ldn[j];
                const R Lu = r < RW - 1 ? L[r + 1][j] : Lup[j];
                kL[r][j] = fL[j] ? t[r][j] * a.wx * fmean<R>(L[r][j], Ll, a.face) : R(0);
                kR[r][j] = fR[j] ? t[r][j] * a.wx * fmean<R>(L[r][j], Lr, a.face) : R(0);
                kD[r][j] = fD ? t[r][j] * a.wy * fmean<R>(L[r][j], Ld, a.face) : R(0);
                kU[r][j] = fU ? t[r][j] * a.wy * fmean<R>(L[r][j], Lu, a.face) : R(0);
            }
        }
        if constexpr (kFloat) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) Lk[r][j] = L[r][j];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                Ldk[j] = Ldn[j];
                Luk[j] = Lup[j];
            }
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
    // from w0 = 0 the first stage is c_0 G (the same number the stage below
    // gives with every difference zero)
    int s0 = 0;
    if (vz) {
        const R cm0 = (R)lane_value(pcm, 0);
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int j = 0; j < C; ++j) v[r][j] = cm0 * G[r][j];
        s0 = 1;
    }
    for (int s = s0; s < Kin; ++s) {
        // the first stage run writes buffer 1 (buffer 0 held the Lambda seams)
        const int buf = (s - s0 + 1) & 1;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            sh_lo[buf][wv][j][lane] = v[0][j];
            sh_hi[buf][wv][j][lane] = v[RW - 1][j];
        }
        __syncthreads();
        R vup[C], ddn[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const R sdn = sh_hi[buf][wdn][j][lane], sup = sh_lo[buf][wup][j][lane];
            const R vdn = wv > 0 ? sdn : v[0][j];
            vup[j] = wv < WAVES - 1 ? sup : v[RW - 1][j];
            ddn[j] = v[0][j] - vdn;
        }
        const double tbd = lane_value(ptb, s);
        const R cm = (R)lane_value(pcm, s), tb = (R)tbd;
        // Each face difference is formed once and shared by the face's two
        // cells: c - c_left is minus the left neighbour's c - c_right, and
        // c - c_below minus the row below's c - c_above (exact in floating
        // point, so S is the same number as with four differences per cell).
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            R drt[C];
#pragma unroll
            for (int j = 0; j < C; ++j) drt[j] = v[r][j] - right_of(v[r], j);
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const R c = v[r][j];
                const R up = r < RW - 1 ? v[r + 1][j] : vup[j];
                const R dlf = -left_of(drt, j);
                const R dup = c - up;
                const R S = kL[r][j] * dlf + kR[r][j] * drt[j] + kD[r][j] * ddn[j] + kU[r][j] * dup;
                R Gr;
                if constexpr (kGinLds) Gr = sG[wv * RW + r][j][lane];
                else Gr = G[r][j];
                v[r][j] = cm * (Gr + tb * c - S);
                ddn[j] = -dup;
            }
        }
        // the output cells are exact after every stage: keep the intermediate
        // stages when asked (the adjoint's recomputation)
        if (kKeep && s + 1 < K) {
            R* dst = a.stages + (int64_t)(s + 1) * a.sstride;
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j)
                    if (xo[j] && yout(r)) dst[(int64_t)(yg0 + r) * a.nx + xg[j]] = v[r][j];
        }
    }
    // Final stage (b = 0) of the FP32 correction form, in double on v = g + w:
    // T = g - tau rC64 sum_f w_f mean(Lambda'_a, Lambda'_b) (v_a - v_b), with
    // Lambda' the float conductivities, into Tfin (every cell of the tile:
    // exact K - 1 in from the edge); gfin holds g, rcfin rC64.
    double Tfin[RW][C], gfin[RW][C], rcfin[RW][C];
    if constexpr (kFloat) {
        if (fin) {
            __shared__ double dsh_lo[WAVES][C][64], dsh_hi[WAVES][C][64];
            double vf[RW][C];
#pragma unroll
            for (int r = 0; r < RW; ++r) ld(a.g64, row_at(r), gfin[r]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) vf[r][j] = gfin[r][j] + (double)v[r][j];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                dsh_lo[wv][j][lane] = vf[0][j];
                dsh_hi[wv][j][lane] = vf[RW - 1][j];
            }
            __syncthreads();
            double vup[C], prev[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                prev[j] = wv > 0 ? dsh_hi[wv - 1][j][lane] : vf[0][j];
                vup[j] = wv < WAVES - 1 ? dsh_lo[wv + 1][j][lane] : vf[RW - 1][j];
            }
            const double wxd = a.g64w[0], wyd = a.g64w[1];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int y = yg0 + r;
                const bool iny = y >= 0 && y < a.ny;
                const bool fD = a.pery ? a.ny > 1 : (iny && y > 0);
                const bool fU = a.pery ? a.ny > 1 : (iny && y < a.ny - 1);
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    const double c = vf[r][j];
                    const double up = r < RW - 1 ? vf[r + 1][j] : vup[j];
                    const double La = (double)Lk[r][j];
                    const double Ll = (double)left_of(Lk[r], j), Lr = (double)right_of(Lk[r], j);
                    const double Ld = (double)(r > 0 ? Lk[r - 1][j] : Ldk[j]);
                    const double Lu = (double)(r < RW - 1 ? Lk[r + 1][j] : Luk[j]);
                    const double lf = left_of(vf[r], j), rt = right_of(vf[r], j);
                    double S = 0.0;
                    if (fL[j]) S += wxd * fmean<double>(La, Ll, a.face) * (c - lf);
                    if (fR[j]) S += wxd * fmean<double>(La, Lr, a.face) * (c - rt);
                    if (fD) S += wyd * fmean<double>(La, Ld, a.face) * (c - prev[j]);
                    if (fU) S += wyd * fmean<double>(La, Lu, a.face) * (c - up);
                    prev[j] = c;
                    Tfin[r][j] = S;
                }
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) ld(a.rC64, row_at(r), rcfin[r]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) Tfin[r][j] = gfin[r][j] - a.taud * rcfin[r][j] * Tfin[r][j];
            if (a.lam_next) {
                // Coefficients of the next Picard pass at the new iterate T
                // (valid K cells in from the edge; g = T^n): the conductivity
                // in double for the bound, its float rounding and the source
                // q = -tau rC' D' g from the float-rounded Lambda' and rC', at
                // the output cells (K+1 in), faces in the order -x, +x, -y, +y.
                double Ln[RW][C], a2v[RW][C], m1v[RW][C], m2v[RW][C];
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int64_t o = row_at(r);
                    ld(a.alpha2, o, a2v[r]);
                    if constexpr (kSH) {
                        ld(a.m1, o, m1v[r]);
                        ld(a.m2, o, m2v[r]);
                    } else {
#pragma unroll
                        for (int j = 0; j < C; ++j) m1v[r][j] = m2v[r][j] = 0.0;
                    }
                }
#pragma unroll
                for (int r = 0; r < RW; ++r)
#pragma unroll
                    for (int j = 0; j < C; ++j) {
                        const double tn = Tfin[r][j];
                        Ln[r][j] = law(tn, a2v[r][j], m1v[r][j], m2v[r][j]);
                    }
                __shared__ double esh[4][WAVES][C][64];  // seams of Lambda and g
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    esh[0][wv][j][lane] = Ln[0][j];
                    esh[1][wv][j][lane] = Ln[RW - 1][j];
                    esh[2][wv][j][lane] = gfin[0][j];
                    esh[3][wv][j][lane] = gfin[RW - 1][j];
                }
                __syncthreads();
                double Ldn[C], Lup[C], gdn[C], gup[C];
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    Ldn[j] = wv > 0 ? esh[1][wv - 1][j][lane] : Ln[0][j];
                    Lup[j] = wv < WAVES - 1 ? esh[0][wv + 1][j][lane] : Ln[RW - 1][j];
                    gdn[j] = wv > 0 ? esh[3][wv - 1][j][lane] : gfin[0][j];
                    gup[j] = wv < WAVES - 1 ? esh[2][wv + 1][j][lane] : gfin[RW - 1][j];
                }
                double bound = 0.0;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    float Lf[C];
#pragma unroll
                    for (int j = 0; j < C; ++j) Lf[j] = (float)Ln[r][j];
#pragma unroll
                    for (int j = 0; j < C; ++j) {
                        const double L = Ln[r][j];
                        const double Ll = left_of(Ln[r], j), Lr = right_of(Ln[r], j);
                        const float Llf = left_of(Lf, j), Lrf = right_of(Lf, j);
                        const double gl = left_of(gfin[r], j), gr = right_of(gfin[r], j);
                        const double Ld = r > 0 ? Ln[r - 1][j] : Ldn[j], Lu = r < RW - 1 ? Ln[r + 1][j] : Lup[j];
                        const double gd = r > 0 ? gfin[r - 1][j] : gdn[j], gu = r < RW - 1 ? gfin[r + 1][j] : gup[j];
                        const int y = yg0 + r;
                        if (xo[j] && yout(r)) {
                            const bool fD = a.pery ? a.ny > 1 : y > 0;
                            const bool fU = a.pery ? a.ny > 1 : y < a.ny - 1;
                            const int64_t o = (int64_t)y * a.nx + xg[j];
                            double d = 0.0;
                            if (fL[j]) d += wxd * fmean<double>(L, Ll, a.face);
                            if (fR[j]) d += wxd * fmean<double>(L, Lr, a.face);
                            if (fD) d += wyd * fmean<double>(L, Ld, a.face);
                            if (fU) d += wyd * fmean<double>(L, Lu, a.face);
                            bound = fmax(bound, 2.0 * d * rcfin[r][j]);
                            const double La = (double)Lf[j], rf = (double)(float)rcfin[r][j], ga = gfin[r][j];
                            double Sq = 0.0;
                            if (fL[j]) Sq += wxd * fmean<double>(La, (double)Llf, a.face) * (ga - gl);
                            if (fR[j]) Sq += wxd * fmean<double>(La, (double)Lrf, a.face) * (ga - gr);
                            if (fD) Sq += wyd * fmean<double>(La, (double)(float)Ld, a.face) * (ga - gd);
                            if (fU) Sq += wyd * fmean<double>(La, (double)(float)Lu, a.face) * (ga - gu);
                            a.Lam32_next[o] = Lf[j];
                            a.q32_next[o] = (float)(-a.taud * rf * Sq);
                        }
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
    // any is used (bit r*C + j of outm: cell j of row r of this lane is an
    // output cell).  The double kernels read them row by row: there the
    // registers that batching takes cost more than the load order gains
    // (measured).
    unsigned outm = 0;
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < C; ++j)
            if (xo[j] && yout(r)) outm |= 1u << (r * C + j);
    auto out_at = [&](int r, int j) -> int64_t {
        return (outm >> (r * C + j)) & 1u ? (int64_t)(yg0 + r) * a.nx + xg[j] : 0;
    };
    double titv[RW][C];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < C; ++j) titv[r][j] = 0.0;
    if constexpr (kFloat) {
        if (a.Tit && a.ps.dmax && !tit_is_g) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) titv[r][j] = a.Tit[out_at(r, j)];
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < C; ++j) {
            if ((outm >> (r * C + j)) & 1u) {
                const int64_t o = (int64_t)(yg0 + r) * a.nx + xg[j];
                double tnew;
                if (fin) {
                    tnew = Tfin[r][j];
                    a.out64[o] = tnew;
                } else {
                    a.out[o] = v[r][j];
                    tnew = (double)v[r][j];
                }
                if (a.Tit) {
                    const double tn = tnew;
                    // the Picard change only where asked for (ps.dmax set)
                    if (a.ps.dmax) {
                        double tit;
                        if (tit_is_g) {
                            if constexpr (kFloat) tit = gfin[r][j];
                            else tit = (double)sG[wv * RW + r][j][lane];
                        } else {
                            if constexpr (kFloat) tit = titv[r][j];
                            else tit = a.Tit[o];
                        }
                        dmax = fmax(dmax, fabs(tn - tit));
                    }
                    tmax = fmax(tmax, fabs(tn));
                    if (!(tn > 0.0) || isinf(tn)) bad += 1.0;
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
            if (a.ps.dmax)
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
            // With next_step the next step's instead: every cell relaxed from
            // (alpha2, v, v, m1, m2) first, Lambda at the relaxed state.
            const bool next_step = a.next_step != 0;
            // The partial densities enter only the relaxation of interface
            // cells (pure cells keep their T and alpha2) and the Spitzer-Harm
            // law; 1/C, which they also fix, is the step's own (equal p_inf),
            // so under the power law they are read in interface cells only.
            double Ln[RW][C], Tr[RW][C], ar[RW][C];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                double a2v[C], m1[C], m2[C];
                const int64_t o = row_at(r);
                ld(a.alpha2, o, a2v);
                if constexpr (kSH) {
                    ld(a.m1, o, m1);
                    ld(a.m2, o, m2);
                } else if (next_step) {
#pragma unroll
                    for (int j = 0; j < C; ++j) {
                        m1[j] = m2[j] = 0.0;
                        if (phys::is_mixed(a2v[j], a.eps)) {
                            const int64_t oj = o + (sel[j] ? 0 : 1);
                            m1[j] = a.m1[oj];
                            m2[j] = a.m2[oj];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    if (next_step) {
                        phys::relax_cell(a.ph, a.eps, a2v[j], v[r][j], v[r][j], m1[j], m2[j], Tr[r][j], ar[r][j]);
                        Ln[r][j] = law(Tr[r][j], ar[r][j], m1[j], m2[j]);
                    } else if constexpr (kSH) {
                        Ln[r][j] = law(v[r][j], a2v[j], m1[j], m2[j]);
                    } else {
                        Ln[r][j] = law(v[r][j], a2v[j], 0.0, 0.0);
                    }
                }
            }
            // the seam buffer not used by the last stage: its reads all
            // precede that stage's barrier
            const int b2 = (K + 1) & 1;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                sh_lo[b2][wv][j][lane] = Ln[0][j];
                sh_hi[b2][wv][j][lane] = Ln[RW - 1][j];
            }
            __syncthreads();
            double Ldn[C], Lup[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                Ldn[j] = wv > 0 ? sh_hi[b2][wv - 1][j][lane] : Ln[0][j];
                Lup[j] = wv < WAVES - 1 ? sh_lo[b2][wv + 1][j][lane] : Ln[RW - 1][j];
            }
            double bound = 0.0;
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    const double Ll = left_of(Ln[r], j), Lr = right_of(Ln[r], j);
                    const double Ld = r > 0 ? Ln[r - 1][j] : Ldn[j];
                    const double Lu = r < RW - 1 ? Ln[r + 1][j] : Lup[j];
                    const int y = yg0 + r;
                    if (xo[j] && yout(r)) {
                        const bool fD = a.pery ? a.ny > 1 : y > 0;
                        const bool fU = a.pery ? a.ny > 1 : y < a.ny - 1;
                        const int64_t o = (int64_t)y * a.nx + xg[j];
                        double d = 0.0;
                        if (fL[j]) d += a.wx * fmean<double>(Ln[r][j], Ll, a.face);
                        if (fR[j]) d += a.wx * fmean<double>(Ln[r][j], Lr, a.face);
                        if (fD) d += a.wy * fmean<double>(Ln[r][j], Ld, a.face);
                        if (fU) d += a.wy * fmean<double>(Ln[r][j], Lu, a.face);
                        const double rc = a.rC[o];
                        bound = fmax(bound, 2.0 * d * rc);
                        a.Lam_next[o] = Ln[r][j];
                        if (next_step) {
                            a.Tn_next[o] = Tr[r][j];
                            a.a2_next[o] = ar[r][j];
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
                double* out64 = nullptr, const NextCoef* nc = nullptr, int vzero = 0) {
    TBArgs<R> a{};
    a.vzero = vzero;
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
    // two cells per lane (float stages only): a lane's pair must not
    // straddle a periodic wrap
    constexpr bool kWideOk = sizeof(R) == 4;
    const bool wide = kWideOk && tall && g.nx >= WIDE_COLS && (g.nx % 2 == 0 || !g.per[0]);
    const int kmax = tall ? KMAX_TB : KMAX_SHORT;
    const int EXT_X = wide ? 128 : 64;
    const int EXT_Y = wide ? 16 * (ROWS / 2) : (tall ? 16 : 8) * ROWS;
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
    a.hx = wide ? (a.H + 1) & ~1 : a.H;
    a.ox = EXT_X - 2 * a.hx;
    a.oy = EXT_Y - 2 * a.H;
    a.tiles_x = (g.nx + a.ox - 1) / a.ox;
    int tiles_y = (g.ny + a.oy - 1) / a.oy;
    for (int k = 0; k < K; ++k) {
        if (st.lam) a.chat[k] = st.chat[k];
        else a.tb[k] = st.tb[k];
    }
    const dim3 grid((unsigned)(a.tiles_x * tiles_y));
    const bool sh = nc && nc->ph.spitzer;
    auto go = [&](auto kern, int nw) { hipLaunchKernelGGL(kern, grid, dim3(64 * nw), 0, s, a); };
    if (stages) {  // (no epilogue: the kept-stage launches of the adjoint's recompute)
        if (tall) go(k_tb2d<R, 16, 1, true, false>, 16);
        else go(k_tb2d<R, 8, 1, true, false>, 8);
    } else if (sh) {
        if constexpr (kWideOk) {
            if (wide) {
                go(k_tb2d<R, 16, 2, false, true>, 16);
                return K;
            }
        }
        if (tall) go(k_tb2d<R, 16, 1, false, true>, 16);
        else go(k_tb2d<R, 8, 1, false, true>, 8);
    } else {
        if constexpr (kWideOk) {
            if (wide) {
                go(k_tb2d<R, 16, 2, false, false>, 16);
                return K;
            }
        }
        if (tall) go(k_tb2d<R, 16, 1, false, false>, 16);
        else go(k_tb2d<R, 8, 1, false, false>, 8);
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
                    const NextCoef* nc, bool* nc_done, bool w_zero) {
    if (nc_done) *nc_done = false;
    if (use_tb2d(g, count)) {
        if (last) {
            if (nc_done) *nc_done = nc != nullptr;
            return launch_tb2d<float>(s, g, face, w, qn, Lam32, rC32, nullptr, st, count, tau, Tit, ps, nullptr, 0,
                                      rhs, rC, out64, nc, w_zero ? 1 : 0);
        }
        return launch_tb2d<float>(s, g, face, w, qn, Lam32, rC32, out, st, count, tau, nullptr, PassSlots{}, nullptr,
                                  0, nullptr, nullptr, nullptr, nullptr, w_zero ? 1 : 0);
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
