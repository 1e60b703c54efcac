// One LIM stage (eq. LIM; with b = 0 the final stage, eq. LIM_last) on 3D
// grids, marching along z.
//
// A wave owns 64 consecutive x cells (one per lane) by ROWS consecutive y
// rows and a chunk of z planes.  It walks the chunk plane by plane, keeping
// v and Lambda of the previous, current and next plane for its rows and the
// two rows around them in registers: the z- and y-neighbours of a cell are
// the lane's own registers, the x-neighbours come from the adjacent lanes
// (DPP), and the two lanes at the ends of the wave load the x-halo cell of
// their row.  Every value is read from memory once per plane and chunk (the
// extra y rows and z planes of the window are the only re-reads), and waves
// never wait on each other: no LDS, no barrier.
//
// Arithmetic as the one-stage kernels: S = sum_f w_f mean(Lambda_a,
// Lambda_b) (v_a - v_b) over the faces -x, +x, -y, +y, -z, +z, then
// out = c_m (G + tau b_m v - tau rC S); in FP32 contexts v is the correction
// w and G the correction source q, in float.
#include <hip/hip_runtime.h>

#include "tlim_device.h"
#include "tlim_sweep.h"

namespace tlim {

namespace {

using tb::fmean;
using tb::fold;
using tb::from_left;
using tb::from_right;

constexpr int kZWaves = 4;

template <typename R>
struct Z3Args {
    const R* v;
    const R* G;
    const R* Lam;
    const R* rC;
    R* out;
    StageParam sp;
    double tau;
    const double* Tit;  // FP64 final stage: accumulate the pass reductions into ps
    PassSlots ps;
    int nx, ny, nz, perx, pery, perz;
    double wx, wy, wz;
    int face, tiles_x, tiles_y, zc, nwaves;
    // kCorr (R = double): the final stage of the FP32 correction form, on
    // v = G + w32 with the float conductivities Lam32 (G = g, rC = 1/C in
    // double); v and Lam are then unused
    const float* w32;
    const float* Lam32;
    // kFromG: the input is the stage before this one from w = 0, c_0 G
    // (c_0 = 1/(1 + tau b_0) of sp_in), read from G; v is then unused
    StageParam sp_in;
};

template <typename R, int ROWS, bool kCorr, bool kFromG = false>
__global__ void __launch_bounds__(64 * kZWaves) k_z3d(Z3Args<R> a) {
    constexpr int RW = ROWS + 2;
    const int lane = threadIdx.x & 63;
    const int wid = tb::xcd_block() * kZWaves + (threadIdx.x >> 6);  // waves in XCD order
    // tau*b of the stage (every lane of every wave takes part in the fold)
    double tbd = a.sp.tb;
    if (a.sp.lam) {
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) m = fmax(m, a.sp.lam[lane + 64 * k]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        tbd = a.tau * m * a.sp.chat;
    }
    // the input's scale: 1, or c_0 of the stage folded into this one (the
    // same number that stage's cm was)
    R vs = R(1);
    if constexpr (kFromG) {
        double tb0 = a.sp_in.tb;
        if (a.sp_in.lam) {
            double m = 0.0;
#pragma unroll
            for (int k = 0; k < kSlots / 64; ++k) m = fmax(m, a.sp_in.lam[lane + 64 * k]);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
            tb0 = a.tau * m * a.sp_in.chat;
        }
        vs = (R)(1.0 / (1.0 + tb0));
    }
    if (wid >= a.nwaves) return;  // wave-uniform
    const int tx = wid % a.tiles_x, rest = wid / a.tiles_x;
    const int ty = rest % a.tiles_y, tz = rest / a.tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int xg = tx * 64 + lane;
    const int xi = fold(xg, nx, a.perx);
    const int xl = fold(tx * 64 - 1, nx, a.perx), xr = fold(tx * 64 + 64, nx, a.perx);
    const bool inx = xg < nx;
    const bool fL = a.perx ? nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? nx > 1 : (inx && xg < nx - 1);
    const int y0 = ty * ROWS, z0 = tz * a.zc;
    const int z1 = z0 + a.zc < nz ? z0 + a.zc : nz;
    const R cm = (R)(1.0 / (1.0 + tbd)), tb = (R)tbd, tf = (R)a.tau;
    const R wx = (R)a.wx, wy = (R)a.wy, wz = (R)a.wz;
    const int face = a.face;

    // 32-bit element offsets (the launcher requires N < 2^32): global loads
    // then take a scalar base and one VGPR offset
    unsigned rowoff[RW];  // y offsets of the window rows within a plane
#pragma unroll
    for (int r = 0; r < RW; ++r) rowoff[r] = (unsigned)fold(y0 - 1 + r, ny, a.pery) * (unsigned)nx;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned uxi = (unsigned)xi;

    // Software pipeline: while plane z is computed, plane z+2 (and the own
    // cells' G, 1/C and the x-halo of plane z+1) are already being loaded.
    R vm[RW], vc[RW], vp[RW], vq[RW], Lm[RW], Lc[RW], Lp[RW], Lq[RW];
    R Gc[ROWS], rc_c[ROWS], Gn[ROWS], rc_n[ROWS], hvc[ROWS], hLc[ROWS], hvn[ROWS], hLn[ROWS];
    auto ld_v = [&](unsigned i) -> R {
        if constexpr (kCorr) return a.G[i] + (R)a.w32[i];
        else if constexpr (kFromG) return vs * a.G[i];
        else return a.v[i];
    };
    auto ld_L = [&](unsigned i) -> R {
        if constexpr (kCorr) return (R)a.Lam32[i];
        else return a.Lam[i];
    };
    auto load_plane = [&](int z, R* vv, R* LL) {
        const unsigned pz = (unsigned)fold(z, nz, a.perz) * plane;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            vv[r] = ld_v(pz + rowoff[r] + uxi);
            LL[r] = ld_L(pz + rowoff[r] + uxi);
        }
    };
    // own cells of plane z (clamped into the grid: only used for z < z1):
    // G and 1/C, and the x-halo cells of the ends of the wave.  The halo
    // cells of all rows come in one load per field (lane q < ROWS: the left
    // halo of row q, lane ROWS + q: the right one) and go to the end lanes
    // by shuffle.
    const int hq = lane < ROWS ? lane : lane - ROWS;
    const bool hload = lane < 2 * ROWS;
    const unsigned hoff = hload ? (unsigned)fold(y0 + hq, ny, a.pery) * (unsigned)nx + (unsigned)(lane < ROWS ? xl : xr)
                                : 0u;
    auto load_own = [&](int z, R* GG, R* rr, R* hv, R* hL) {
        const unsigned pz = (unsigned)(z < nz ? z : nz - 1) * plane;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            GG[r] = a.G[pz + rowoff[r + 1] + uxi];
            rr[r] = a.rC[pz + rowoff[r + 1] + uxi];
        }
        const R hvq = hload ? ld_v(pz + hoff) : R(0);
        const R hLq = hload ? ld_L(pz + hoff) : R(0);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int src = lane == 63 ? ROWS + r : r;
            hv[r] = __shfl(hvq, src, 64);
            hL[r] = __shfl(hLq, src, 64);
        }
    };
    load_plane(z0 - 1, vm, Lm);
    load_plane(z0, vc, Lc);
    load_plane(z0 + 1, vp, Lp);
    load_own(z0, Gc, rc_c, hvc, hLc);
    double dmax = 0.0, tmax = 0.0, bad = 0.0;
    for (int z = z0; z < z1; ++z) {
        const unsigned pc = (unsigned)z * plane;
        load_plane(z + 2, vq, Lq);
        load_own(z + 1, Gn, rc_n, hvn, hLn);
        // x-neighbours of the current plane, with every lane active
        R vl[ROWS], vr[ROWS], Ll[ROWS], Lr[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            vl[r] = from_left(vc[r + 1]);
            vr[r] = from_right(vc[r + 1]);
            Ll[r] = from_left(Lc[r + 1]);
            Lr[r] = from_right(Lc[r + 1]);
            if (lane == 0) {
                vl[r] = hvc[r];
                Ll[r] = hLc[r];
            }
            if (lane == 63) {
                vr[r] = hvc[r];
                Lr[r] = hLc[r];
            }
        }
        const bool fB = a.perz ? nz > 1 : z > 0;
        const bool fF = a.perz ? nz > 1 : z < nz - 1;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = y0 + r;
            if (inx && y < ny) {
                const bool fD = a.pery ? ny > 1 : y > 0;
                const bool fU = a.pery ? ny > 1 : y < ny - 1;
                const R c = vc[r + 1], La = Lc[r + 1];
                R S = R(0);
                if (fL) S += wx * fmean<R>(La, Ll[r], face) * (c - vl[r]);
                if (fR) S += wx * fmean<R>(La, Lr[r], face) * (c - vr[r]);
                if (fD) S += wy * fmean<R>(La, Lc[r], face) * (c - vc[r]);
                if (fU) S += wy * fmean<R>(La, Lc[r + 2], face) * (c - vc[r + 2]);
                if (fB) S += wz * fmean<R>(La, Lm[r + 1], face) * (c - vm[r + 1]);
                if (fF) S += wz * fmean<R>(La, Lp[r + 1], face) * (c - vp[r + 1]);
                const unsigned o = pc + (unsigned)y * (unsigned)nx + (unsigned)xg;
                const R t = cm * (Gc[r] + tb * c - tf * rc_c[r] * S);
                a.out[o] = t;
                if (a.Tit) {
                    const double tn = (double)t;
                    if (a.ps.dmax) dmax = fmax(dmax, fabs(tn - a.Tit[o]));
                    tmax = fmax(tmax, fabs(tn));
                    if (!(tn > 0.0) || isinf(tn)) bad += 1.0;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            vm[r] = vc[r];
            Lm[r] = Lc[r];
            vc[r] = vp[r];
            Lc[r] = Lp[r];
            vp[r] = vq[r];
            Lp[r] = Lq[r];
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            Gc[r] = Gn[r];
            rc_c[r] = rc_n[r];
            hvc[r] = hvn[r];
            hLc[r] = hLn[r];
        }
    }
    if (a.Tit) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
            tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
            bad += __shfl_xor(bad, o, 64);
        }
        if (lane == 0) {
            const int sl = wid % kSlots;
            if (a.ps.dmax)
                atomicMax((unsigned long long*)(a.ps.dmax + sl), (unsigned long long)__double_as_longlong(dmax + 0.0));
            atomicMax((unsigned long long*)(a.ps.tmax + sl), (unsigned long long)__double_as_longlong(tmax + 0.0));
            if (bad != 0.0) atomicAdd(a.ps.bad + sl, bad);
        }
    }
}

// y rows per wave: fewer in double, to keep two waves per SIMD
template <typename R>
constexpr int z_rows() {
    return sizeof(R) == 8 ? 4 : 8;
}


template <typename R, bool kCorr, bool kFromG = false>
void launch_z3d_impl(hipStream_t s, const DevGrid& g, int face, const R* v, const R* G, const R* Lam, const R* rC,
                     R* out, StageParam sp, double tau, const double* Tit, PassSlots ps, const float* w32,
                     const float* Lam32, StageParam sp_in = StageParam{nullptr, 0.0, 0.0}) {
    Z3Args<R> a{};
    a.sp_in = sp_in;
    a.w32 = w32;
    a.Lam32 = Lam32;
    a.v = v;
    a.G = G;
    a.Lam = Lam;
    a.rC = rC;
    a.out = out;
    a.sp = sp;
    a.tau = tau;
    a.Tit = Tit;
    a.ps = ps;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.perz = g.per[2];
    a.wx = g.w[0];
    a.wy = g.w[1];
    a.wz = g.w[2];
    a.face = face;
    a.tiles_x = (g.nx + 63) / 64;
    constexpr int rows = z_rows<R>();
    a.tiles_y = (g.ny + rows - 1) / rows;
    // z chunks sized for about 2048 (float) or 4096 (double) waves, 4..64
    // planes each: fewer, longer chunks re-read fewer halo planes (at 256^3
    // the float stage takes 83 us with 2048 waves, 88 us with 4096 and
    // 128 us with 1024, where too few waves stay in flight)
    const int64_t cols = (int64_t)a.tiles_x * a.tiles_y;
    int64_t zc = (int64_t)g.nz * cols / (sizeof(R) == 4 ? 2048 : 4096);
    zc = zc < 4 ? 4 : (zc > 64 ? 64 : zc);
    a.zc = (int)zc;
    const int64_t nw = cols * ((g.nz + a.zc - 1) / a.zc);
    a.nwaves = (int)nw;
    const unsigned blocks = (unsigned)((nw + kZWaves - 1) / kZWaves);
    hipLaunchKernelGGL((k_z3d<R, rows, kCorr, kFromG>), dim3(blocks), dim3(64 * kZWaves), 0, s, a);
}

}  // namespace

template <typename R>
void launch_z3d(hipStream_t s, const DevGrid& g, int face, const R* v, const R* G, const R* Lam, const R* rC, R* out,
                StageParam sp, double tau, const double* Tit, PassSlots ps) {
    launch_z3d_impl<R, false>(s, g, face, v, G, Lam, rC, out, sp, tau, Tit, ps, nullptr, nullptr);
}

void launch_z3d_two_from_zero32(hipStream_t s, const DevGrid& g, int face, const float* qn, const float* Lam32,
                                const float* rC32, float* out, StageParam sp0, StageParam sp1, double tau) {
    launch_z3d_impl<float, false, true>(s, g, face, nullptr, qn, Lam32, rC32, out, sp1, tau, nullptr, PassSlots{},
                                        nullptr, nullptr, sp0);
}

void launch_z3d_final32(hipStream_t s, const DevGrid& g, int face, const float* w, const double* rhs,
                        const float* Lam32, const double* rC, double* out, double tau, const double* Tit,
                        PassSlots ps) {
    launch_z3d_impl<double, true>(s, g, face, nullptr, rhs, nullptr, rC, out, StageParam{nullptr, 0.0, 0.0}, tau, Tit,
                                  ps, w, Lam32);
}

bool use_z3d(const DevGrid& g) { return g.nz > 1 && g.N < ((int64_t)1 << 32); }

template void launch_z3d<double>(hipStream_t, const DevGrid&, int, const double*, const double*, const double*,
                                 const double*, double*, StageParam, double, const double*, PassSlots);
template void launch_z3d<float>(hipStream_t, const DevGrid&, int, const float*, const float*, const float*,
                                const float*, float*, StageParam, double, const double*, PassSlots);

}  // namespace tlim

// ------------------------------------------------------------------ adjoint

namespace tlim {

namespace {

// One reverse stage of the LIM adjoint on a 3D grid in psi = C^-1 lambda
// form (arithmetic face means), marching along z like k_z3d:
//   psi^(m-1) = c_m (tau b_m psi^(m) - tau rC sum_f w_f Lambda_f (psi_a - psi_b)),
//   dgpsi += c_m psi^(m)_a,
//   gLam  += c_m sum_f (tau w_f / 2) (v_b - v_a)^(m-1) (psi_a - psi_b)^(m),
// the same operations as the blocked 2D reverse stages (tlim_adjoint.hip)
// with the z faces added.  A wave keeps psi, v^(m-1) and Lambda of four
// consecutive planes for its rows and the rows around them in registers.
struct AZ3Args {
    const double* psi;
    const double* vprev;
    const double* Lam;
    const double* rC;
    double* psi_out;
    double* dgpsi;
    double* gLam;
    double cm, tb, tau;
    int nx, ny, nz, perx, pery, perz;
    double wx, wy, wz;
    int tiles_x, tiles_y, zc, nwaves;
};

template <int ROWS>
__global__ void __launch_bounds__(64 * kZWaves) k_adj_z3d(AZ3Args a) {
    constexpr int RW = ROWS + 2;
    const int lane = threadIdx.x & 63;
    // launch order: the z-marching reverse stage measured 2% slower in XCD order
    const int wid = blockIdx.x * kZWaves + (threadIdx.x >> 6);
    if (wid >= a.nwaves) return;  // wave-uniform
    const int tx = wid % a.tiles_x, rest = wid / a.tiles_x;
    const int ty = rest % a.tiles_y, tz = rest / a.tiles_y;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int xg = tx * 64 + lane;
    const int xi = fold(xg, nx, a.perx);
    const int xl = fold(tx * 64 - 1, nx, a.perx), xr = fold(tx * 64 + 64, nx, a.perx);
    const bool inx = xg < nx;
    const bool fL = a.perx ? nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? nx > 1 : (inx && xg < nx - 1);
    const int y0 = ty * ROWS, z0 = tz * a.zc;
    const int z1 = z0 + a.zc < nz ? z0 + a.zc : nz;
    const double cm = a.cm, tb = a.tb, tf = a.tau;
    const double wx = a.wx, wy = a.wy, wz = a.wz;
    const double hx = 0.5 * tf * wx, hy = 0.5 * tf * wy, hz = 0.5 * tf * wz;

    unsigned rowoff[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) rowoff[r] = (unsigned)fold(y0 - 1 + r, ny, a.pery) * (unsigned)nx;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned uxi = (unsigned)xi;
    // x-halo cells of the end lanes: all rows in one load per field (lane
    // q < ROWS: the left halo of row q, lane ROWS + q: the right one), handed
    // to the end lanes by shuffle
    const int hq = lane < ROWS ? lane : lane - ROWS;
    const bool hload = lane < 2 * ROWS;
    const unsigned hoff = hload ? (unsigned)fold(y0 + hq, ny, a.pery) * (unsigned)nx + (unsigned)(lane < ROWS ? xl : xr)
                                : 0u;

    // windows: p (psi), u (v^(m-1)), L (Lambda) of planes z-1 (m), z (c),
    // z+1 (p), z+2 (q)
    double pm[RW], pc[RW], pp[RW], pq[RW], um[RW], uc[RW], up_[RW], uq[RW], Lm[RW], Lc[RW], Lp[RW], Lq[RW];
    // own cells of planes z (c) and z+1 (n): 1/C, the accumulators, and the
    // x-halo cells of the end lanes
    double rcc[ROWS], dgc[ROWS], glc[ROWS], rcn[ROWS], dgn[ROWS], gln[ROWS];
    double hpc[ROWS], huc[ROWS], hLc[ROWS], hpn[ROWS], hun[ROWS], hLn[ROWS];
    auto load_plane = [&](int z, double* P, double* U, double* L) {
        const unsigned pz = (unsigned)fold(z, nz, a.perz) * plane;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            P[r] = a.psi[pz + rowoff[r] + uxi];
            U[r] = a.vprev[pz + rowoff[r] + uxi];
            L[r] = a.Lam[pz + rowoff[r] + uxi];
        }
    };
    auto load_own = [&](int z, double* rc, double* dg, double* gl, double* hp, double* hu, double* hL) {
        const unsigned pz = (unsigned)(z < nz ? z : nz - 1) * plane;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const unsigned o = pz + rowoff[r + 1] + uxi;
            rc[r] = a.rC[o];
            dg[r] = a.dgpsi[o];
            gl[r] = a.gLam[o];
        }
        const double hpq = hload ? a.psi[pz + hoff] : 0.0;
        const double huq = hload ? a.vprev[pz + hoff] : 0.0;
        const double hLq = hload ? a.Lam[pz + hoff] : 0.0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int src = lane == 63 ? ROWS + r : r;
            hp[r] = __shfl(hpq, src, 64);
            hu[r] = __shfl(huq, src, 64);
            hL[r] = __shfl(hLq, src, 64);
        }
    };
    load_plane(z0 - 1, pm, um, Lm);
    load_plane(z0, pc, uc, Lc);
    load_plane(z0 + 1, pp, up_, Lp);
    load_own(z0, rcc, dgc, glc, hpc, huc, hLc);
    for (int z = z0; z < z1; ++z) {
        const unsigned pzc = (unsigned)z * plane;
        load_plane(z + 2, pq, uq, Lq);
        load_own(z + 1, rcn, dgn, gln, hpn, hun, hLn);
        const bool fB = a.perz ? nz > 1 : z > 0;
        const bool fF = a.perz ? nz > 1 : z < nz - 1;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            // x-neighbours with every lane active
            double pl = from_left(pc[r + 1]), pr = from_right(pc[r + 1]);
            double ul = from_left(uc[r + 1]), ur = from_right(uc[r + 1]);
            double Ll = from_left(Lc[r + 1]), Lr = from_right(Lc[r + 1]);
            if (lane == 0) {
                pl = hpc[r];
                ul = huc[r];
                Ll = hLc[r];
            }
            if (lane == 63) {
                pr = hpc[r];
                ur = huc[r];
                Lr = hLc[r];
            }
            const int y = y0 + r;
            if (inx && y < ny) {
                const bool fD = a.pery ? ny > 1 : y > 0;
                const bool fU = a.pery ? ny > 1 : y < ny - 1;
                const double c = pc[r + 1], va = uc[r + 1], La = Lc[r + 1];
                double S = 0.0, G = 0.0;
                if (fL) {
                    S += wx * fmean<double>(La, Ll, 0) * (c - pl);
                    G += hx * (ul - va) * (c - pl);
                }
                if (fR) {
                    S += wx * fmean<double>(La, Lr, 0) * (c - pr);
                    G += hx * (ur - va) * (c - pr);
                }
                if (fD) {
                    S += wy * fmean<double>(La, Lc[r], 0) * (c - pc[r]);
                    G += hy * (uc[r] - va) * (c - pc[r]);
                }
                if (fU) {
                    S += wy * fmean<double>(La, Lc[r + 2], 0) * (c - pc[r + 2]);
                    G += hy * (uc[r + 2] - va) * (c - pc[r + 2]);
                }
                if (fB) {
                    S += wz * fmean<double>(La, Lm[r + 1], 0) * (c - pm[r + 1]);
                    G += hz * (um[r + 1] - va) * (c - pm[r + 1]);
                }
                if (fF) {
                    S += wz * fmean<double>(La, Lp[r + 1], 0) * (c - pp[r + 1]);
                    G += hz * (up_[r + 1] - va) * (c - pp[r + 1]);
                }
                const unsigned o = pzc + (unsigned)y * (unsigned)nx + (unsigned)xg;
                a.psi_out[o] = cm * (tb * c - tf * rcc[r] * S);
                a.dgpsi[o] = dgc[r] + cm * c;
                a.gLam[o] = glc[r] + cm * G;
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            pm[r] = pc[r];
            um[r] = uc[r];
            Lm[r] = Lc[r];
            pc[r] = pp[r];
            uc[r] = up_[r];
            Lc[r] = Lp[r];
            pp[r] = pq[r];
            up_[r] = uq[r];
            Lp[r] = Lq[r];
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            rcc[r] = rcn[r];
            dgc[r] = dgn[r];
            glc[r] = gln[r];
            hpc[r] = hpn[r];
            huc[r] = hun[r];
            hLc[r] = hLn[r];
        }
    }
}

constexpr int kAdjRows = 2;

__global__ void __launch_bounds__(256) k_scale_rc(int64_t n, const double* __restrict__ x, const double* __restrict__ rC,
                                                  double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * rC[i];
}

}  // namespace

bool use_adj_z3d(const DevGrid& g, int face) { return use_z3d(g) && face == 0; }

void launch_psi_from_lambda(hipStream_t s, int64_t n, const double* lam, const double* rC, double* psi) {
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_scale_rc, dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, s, n, lam, rC, psi);
}

void launch_adj_z3d(hipStream_t s, const DevGrid& g, const double* psi, const double* vprev, const double* Lam,
                    const double* rC, double* psi_out, double* dgpsi, double* gLam, double cm, double tb,
                    double tau) {
    AZ3Args a{};
    a.psi = psi;
    a.vprev = vprev;
    a.Lam = Lam;
    a.rC = rC;
    a.psi_out = psi_out;
    a.dgpsi = dgpsi;
    a.gLam = gLam;
    a.cm = cm;
    a.tb = tb;
    a.tau = tau;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.perz = g.per[2];
    a.wx = g.w[0];
    a.wy = g.w[1];
    a.wz = g.w[2];
    a.tiles_x = (g.nx + 63) / 64;
    a.tiles_y = (g.ny + kAdjRows - 1) / kAdjRows;
    const int64_t cols = (int64_t)a.tiles_x * a.tiles_y;
    int64_t zc = (int64_t)g.nz * cols / 4096;
    zc = zc < 4 ? 4 : (zc > 64 ? 64 : zc);
    a.zc = (int)zc;
    const int64_t nw = cols * ((g.nz + a.zc - 1) / a.zc);
    a.nwaves = (int)nw;
    const unsigned blocks = (unsigned)((nw + kZWaves - 1) / kZWaves);
    hipLaunchKernelGGL(k_adj_z3d<kAdjRows>, dim3(blocks), dim3(64 * kZWaves), 0, s, a);
}

}  // namespace tlim
