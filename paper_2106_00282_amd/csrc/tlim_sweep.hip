// Inner LIM stages (eq. LIM) with temporal blocking for 2D grids.
//
// One stage of eq. LIM is a 5-point explicit update,
//   v^(m)_a = c_m (G_a + tau b_m v^(m-1)_a - sum_f kappa_af (v^(m-1)_a - v^(m-1)_f)),
//   kappa_af = tau / C_a * w_f * Lambda_f,
// with G = g = T^n + tau f (FP64 form) or G = -tau A' g (FP32 correction form,
// where v is the correction w = v - g).  The final stage (b = 0) of the FP64
// form is the same update with c = 1.
//
// k_tb2d advances K <= KMAX stages per launch.  A workgroup of WAVES wave64s
// loads a 64 x (WAVES*ROWS) extended tile once (v, G, Lambda, 1/C; one
// coalesced 64-wide row per wave per field), builds the four kappa of every
// cell in registers, and then runs the K stages out of registers:
//   - x-neighbours come from the adjacent lanes through DPP wave shifts;
//   - y-neighbours are the lane's own registers (each lane owns ROWS
//     consecutive cells of one column), except at the seams between waves,
//     which go through a double-buffered LDS row (one barrier per stage).
// Cells within K of the extended tile's edge go stale one ring per stage;
// the inner (64-2K) x (WAVES*ROWS-2K) cells are exact and written out.
// Bytes per launch: 4 words read per extended cell + 1 word written per
// output cell, for K stages.
#include <hip/hip_runtime.h>

#include "tlim_sweep.h"

namespace tlim {

namespace {

constexpr int KMAX = 8;
constexpr int WAVES = 8;
constexpr int ROWS = 8;
constexpr int EXT_Y = WAVES * ROWS;

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
    int nx, ny, perx, pery;
    R wx, wy, tau;
    int K, face, tiles_x, ox, oy;
    double taud;
    double tb[KMAX], chat[KMAX];
};

// Lane i receives lane i-1 (wave_shr:1) or lane i+1 (wave_shl:1); with
// bound_ctrl the lanes at the ends receive 0 (they are halo lanes).
__device__ __forceinline__ int dpp_from_left(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_from_right(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true); }

__device__ __forceinline__ double from_left(double x) {
    return __hiloint2double(dpp_from_left(__double2hiint(x)), dpp_from_left(__double2loint(x)));
}
__device__ __forceinline__ double from_right(double x) {
    return __hiloint2double(dpp_from_right(__double2hiint(x)), dpp_from_right(__double2loint(x)));
}
__device__ __forceinline__ float from_left(float x) { return __int_as_float(dpp_from_left(__float_as_int(x))); }
__device__ __forceinline__ float from_right(float x) { return __int_as_float(dpp_from_right(__float_as_int(x))); }

template <typename R>
__device__ __forceinline__ R fmean(R a, R b, int face) {
    if (face == 1) {
        R s = a + b;
        return s > R(0) ? R(2) * (a * b) / s : R(0);
    }
    return R(0.5) * (a + b);
}

// Index of an unwrapped coordinate: wrap on a periodic axis, clamp on an
// adiabatic one (clamped copies only feed halo cells, whose wall faces
// carry kappa = 0).
__device__ __forceinline__ int fold(int c, int n, int per) {
    if (per) {
        int m = c % n;
        return m < 0 ? m + n : m;
    }
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

template <typename R>
__global__ void __launch_bounds__(64 * WAVES, 4) k_tb2d(TBArgs<R> a) {
    __shared__ R sh_lo[2][WAVES][64];  // row 0 of each wave (the "up" row of the wave below)
    __shared__ R sh_hi[2][WAVES][64];  // row ROWS-1 of each wave (the "down" row of the wave above)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int K = a.K;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int xg = tx * a.ox - K + lane;
    const int yg0 = ty * a.oy - K + wv * ROWS;
    const int xi = fold(xg, a.nx, a.perx);
    const bool inx = xg >= 0 && xg < a.nx;
    const bool fL = a.perx ? a.nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? a.nx > 1 : (inx && xg < a.nx - 1);

    R v[ROWS], G[ROWS], kL[ROWS], kR[ROWS], kD[ROWS], kU[ROWS];
    {
        R L[ROWS], t[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int yi = fold(yg0 + r, a.ny, a.pery);
            const int64_t idx = (int64_t)yi * a.nx + xi;
            v[r] = a.v[idx];
            G[r] = a.G[idx];
            L[r] = a.Lam[idx];
            t[r] = a.tau * a.rC[idx];
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
    }
    // lambda_G of the pass from its accumulator row (every wave folds it)
    double lamv = 0.0;
    if (a.lam) {
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) lamv = fmax(lamv, a.lam[lane + 64 * k]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lamv = fmax(lamv, __shfl_xor(lamv, o, 64));
    }
    // Stage s exchanges the seam rows through LDS buffer (s+1)&1; buffer 0
    // held the Lambda seams, whose reads all precede the first barrier below.
    for (int s = 0; s < K; ++s) {
        const int buf = (s + 1) & 1;
        sh_lo[buf][wv][lane] = v[0];
        sh_hi[buf][wv][lane] = v[ROWS - 1];
        __syncthreads();
        const R vdn = wv > 0 ? sh_hi[buf][wv - 1][lane] : v[0];
        const R vup = wv < WAVES - 1 ? sh_lo[buf][wv + 1][lane] : v[ROWS - 1];
        const double tbd = a.lam ? a.taud * lamv * a.chat[s] : a.tb[s];
        const R cm = (R)(1.0 / (1.0 + tbd)), tb = (R)tbd;
        R prev = vdn;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const R c = v[r];
            const R up = r < ROWS - 1 ? v[r + 1] : vup;
            const R lf = from_left(c), rt = from_right(c);
            const R S = kL[r] * (c - lf) + kR[r] * (c - rt) + kD[r] * (c - prev) + kU[r] * (c - up);
            v[r] = cm * (G[r] + tb * c - S);
            prev = c;
        }
    }
    double dmax = 0.0, tmax = 0.0, bad = 0.0;
    if (lane >= K && lane < 64 - K && xg < a.nx) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int row = wv * ROWS + r;
            const int y = yg0 + r;
            if (row >= K && row < EXT_Y - K && y < a.ny) {
                const int64_t o = (int64_t)y * a.nx + xg;
                a.out[o] = v[r];
                if (a.Tit) {
                    const double tn = (double)v[r];
                    dmax = fmax(dmax, fabs(tn - a.Tit[o]));
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
}

template <typename R>
int launch_tb2d(hipStream_t s, const DevGrid& g, int face, const R* v, const R* G, const R* Lam, const R* rC,
                R* out, Stages st, int count, double tau, const double* Tit, PassSlots ps) {
    TBArgs<R> a{};
    int K = count < KMAX ? count : KMAX;
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
    a.face = face;
    a.ox = 64 - 2 * K;
    a.oy = EXT_Y - 2 * K;
    a.tiles_x = (g.nx + a.ox - 1) / a.ox;
    int tiles_y = (g.ny + a.oy - 1) / a.oy;
    for (int k = 0; k < K; ++k) {
        if (st.lam) a.chat[k] = st.chat[k];
        else a.tb[k] = st.tb[k];
    }
    hipLaunchKernelGGL(k_tb2d<R>, dim3((unsigned)(a.tiles_x * tiles_y)), dim3(64 * WAVES), 0, s, a);
    return K;
}

bool use_tb2d(const DevGrid& g, int count) {
    return g.nz == 1 && g.ny >= EXT_Y / 2 && count >= 2;
}

StageParam one_stage(const Stages& st) {
    StageParam sp;
    sp.lam = st.lam;
    sp.tb = st.lam ? 0.0 : st.tb[0];
    sp.chat = st.lam ? st.chat[0] : 0.0;
    return sp;
}

}  // namespace

int sweeps_per_launch(const DevGrid& g, int count) {
    if (use_tb2d(g, count)) return count < KMAX ? count : KMAX;
    return 1;
}

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, Stages st, int count, bool last, double tau,
                    const double* Tit, PassSlots ps) {
    if (use_tb2d(g, count))
        return launch_tb2d<double>(s, g, face, v, rhs, Lam, rC, out, st, count, tau, last ? Tit : nullptr, ps);
    if (last) {
        // the final stage, b = 0, in flux form
        launch_final64(s, g, face, v, rhs, Lam, rC, out, tau, Tit, ps);
    } else {
        launch_stage64(s, g, face, v, rhs, Lam, rC, out, one_stage(st), tau);
    }
    return 1;
}

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* qn,
                    const float* Lam32, const float* rC32, float* out, Stages st, int count, double tau) {
    if (use_tb2d(g, count))
        return launch_tb2d<float>(s, g, face, w, qn, Lam32, rC32, out, st, count, tau, nullptr, PassSlots{});
    launch_stage32(s, g, face, w, qn, Lam32, rC32, out, one_stage(st), tau);
    return 1;
}

}  // namespace tlim
