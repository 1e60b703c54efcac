// gfx950 kernels of the parabolic sub-step (arXiv 2106.00282, Sec. 3.2 and
// Sec. 3.4): temperature relaxation, coefficients, Gershgorin bound, LIM
// stages in FP64 and in the FP32 correction form, the conservative final
// stage, Picard reductions, cycle-mode residual and the adjoint stage.
//
// Layout: structure of arrays, one dense array per field, x fastest.
// Stencil kernels run one work-item per cell on 64x4 tiles (a wave64 covers
// 64 consecutive x cells, so every load is a coalesced 512 B / 256 B row);
// the temporally blocked sweeps live in tlim_sweep.hip.
// Reductions fold each block's cells and add one atomic per block (max on
// the bit pattern of non-negative doubles, add for sums).
#include <hip/hip_runtime.h>
#include <math.h>

#include "tlim_device.h"
#include "tlim_internal.h"

namespace tlim {

namespace {

using phys::cell_conductivity;
using phys::inv_heat_capacity;
using phys::is_mixed;
using phys::powlaw;
using phys::pressure_stiffness;

constexpr int TX = 64;
constexpr int TY = 4;

// ------------------------------------------------------------------ helpers

template <typename R>
__device__ __forceinline__ R face_mean(R a, R b, int face) {
    if (face == 1) {
        R s = a + b;
        return s > R(0) ? R(2) * (a * b) / s : R(0);
    }
    return R(0.5) * (a + b);
}

template <typename R>
__device__ __forceinline__ R face_partial(R a, R b, int face) {
    if (face == 1) {
        R s = a + b;
        return s > R(0) ? R(2) * b * b / (s * s) : R(0);
    }
    return R(0.5);
}

// Neighbour offsets of cell (i,j,k): for each of the six faces, the linear
// offset to the neighbour and whether the face exists (periodic wrap, no
// face at an adiabatic end or on an axis of one cell).
struct Faces {
    int64_t off[6];
    bool has[6];
};

__device__ __forceinline__ void faces_of(const DevGrid& g, int i, int j, int k, Faces& f) {
    const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int c[3] = {i, j, k};
    const int64_t st[3] = {sx, sy, sz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bool multi = n[d] > 1;
        bool lo = c[d] > 0, hi = c[d] < n[d] - 1;
        f.has[2 * d] = multi && (lo || g.per[d]);
        f.off[2 * d] = lo ? -st[d] : (int64_t)(n[d] - 1) * st[d];
        f.has[2 * d + 1] = multi && (hi || g.per[d]);
        f.off[2 * d + 1] = hi ? st[d] : -(int64_t)(n[d] - 1) * st[d];
    }
}

// S = sum_f w_f Lam_f (v_a - v_b), arithmetic in RA.
template <typename RA, typename RV, typename RL>
__device__ __forceinline__ RA stencil(const DevGrid& g, const Faces& f, int64_t a, const RV* __restrict__ v,
                                      const RL* __restrict__ L, int face) {
    RA va = (RA)v[a], La = (RA)L[a], S = RA(0);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!f.has[q]) continue;
        int64_t b = a + f.off[q];
        S += (RA)g.w[q >> 1] * face_mean<RA>(La, (RA)L[b], face) * (va - (RA)v[b]);
    }
    return S;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block reductions for blocks of a multiple of 64 threads (<= 1024) of any
// shape; the result is valid in the block's first thread.
__device__ __forceinline__ int flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
__device__ __forceinline__ int block_threads() { return blockDim.x * blockDim.y * blockDim.z; }

__device__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    int t = flat_tid(), lane = t & 63, wid = t >> 6, nw = block_threads() >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    v = t < nw ? sh[t] : 0.0;
    if (wid == 0) v = wave_sum(v);
    __syncthreads();
    return v;
}
__device__ double block_max(double v, double* sh) {
    v = wave_max(v);
    int t = flat_tid(), lane = t & 63, wid = t >> 6, nw = block_threads() >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    v = t < nw ? sh[t] : -INFINITY;
    if (wid == 0) v = wave_max(v);
    __syncthreads();
    return v;
}

__device__ __forceinline__ int block_slot() {
    return (int)((blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)) % kSlots);
}
// slot of a wave: blocks and their waves spread over the row
__device__ __forceinline__ int wave_slot() {
    int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    return (int)((b * (block_threads() >> 6) + (flat_tid() >> 6)) % kSlots);
}

// atomicMax on the bit pattern orders non-negative doubles (and lets a NaN
// win); -0 is folded to +0 first.
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    v = v + 0.0;
    atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Max of an accumulator row, computed by every wave on its own (all lanes
// of the wave must call it).
__device__ __forceinline__ double row_max(const double* row) {
    const int lane = flat_tid() & 63;
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < kSlots / 64; ++k) m = fmax(m, row[lane + 64 * k]);
    return wave_max(m);
}

// Per-cell contribution to the pass reductions of a new iterate tn given the
// previous iterate ti: max |tn - ti|, max |tn|, count of tn not finite or <= 0.
struct PassAcc {
    double dmax = 0.0, tmax = 0.0, bad = 0.0;
    __device__ void add(double tn, double ti) {
        dmax = fmax(dmax, fabs(tn - ti));
        tmax = fmax(tmax, fabs(tn));
        if (!(tn > 0.0) || isinf(tn)) bad += 1.0;
    }
    // fold the three values over the block with one barrier, then one
    // atomic per value from the block's first thread
    __device__ void store(const PassSlots& ps) {
        __shared__ double red[3][16];
        double r0 = wave_max(dmax), r1 = wave_max(tmax), r3 = wave_sum(bad);
        const int t = flat_tid(), nw = block_threads() >> 6;
        if ((t & 63) == 0) {
            red[0][t >> 6] = r0;
            red[1][t >> 6] = r1;
            red[2][t >> 6] = r3;
        }
        __syncthreads();
        if (t == 0) {
            for (int w = 1; w < nw; ++w) {
                r0 = fmax(r0, red[0][w]);
                r1 = fmax(r1, red[1][w]);
                r3 += red[2][w];
            }
            const int sl = block_slot();
            if (ps.dmax) atomic_max_nonneg(ps.dmax + sl, r0);
            atomic_max_nonneg(ps.tmax + sl, r1);
            if (r3 != 0.0) atomicAdd(ps.bad + sl, r3);
        }
    }
};

__device__ __forceinline__ void cell_ijk(const DevGrid& g, int64_t a, int& i, int& j, int& k) {
    int64_t nxy = (int64_t)g.nx * g.ny;
    k = (int)(a / nxy);
    int64_t r = a - (int64_t)k * nxy;
    j = (int)(r / g.nx);
    i = (int)(r - (int64_t)j * g.nx);
}

int reduce_blocks(int64_t N) {
    int64_t b = (N + kReduceThreads - 1) / kReduceThreads;
    return (int)(b < kReduceBlocks ? (b > 0 ? b : 1) : kReduceBlocks);
}

dim3 tile_grid(const DevGrid& g) { return dim3((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, g.nz); }

// -------------------------------------------------- temperature relaxation

// Relaxation of every cell (phys::relax_cell) in place; Tn and a2n (each
// nullable) also receive the relaxed T and alpha2.
__global__ void __launch_bounds__(256) k_relax(DevGrid g, DevPhases ph, double eps, double* alpha2,
                                               const double* __restrict__ m1, const double* __restrict__ m2,
                                               double* T1, double* T2, double* Tn, double* a2n) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double T, a2;
        phys::relax_cell(ph, eps, alpha2[a], T1[a], T2[a], m1[a], m2[a], T, a2);
        alpha2[a] = a2;
        T1[a] = T;
        T2[a] = T;
        if (Tn) Tn[a] = T;
        if (a2n) a2n[a] = a2;
    }
}

// ------------------------------------------------------------ coefficients

// Coefficients of a Picard pass and the Gershgorin bound in one pass over
// (T, alpha2).  Every cell of the block's 64x4 tile, and of its one-cell
// halo, evaluates its conductivity (and g) once into LDS; the stencil reads
// the neighbours from there.  Tile and halo positions hold the values of the
// folded (periodic-wrapped, adiabatic-clamped) coordinates, so lookups by
// position are right on periodic axes and unused across walls.
// In FP32 contexts (q32 != NULL) it also writes the correction source
// q = -tau rC' D' g (doubles from the float-rounded Lambda' and rC') and
// w0 = float(Tn - g) of the correction form.
struct CoefIn {
    const double *T, *alpha2, *m1, *m2, *Tn, *src1, *src2;
};

// Coordinate of a tile or halo position: one periodic wrap (exact for every
// position a stencil of the tile reads, which is at most one cell outside
// the grid), then a clamp that keeps the unused positions of partial tiles
// in bounds.
__device__ __forceinline__ int fold_coord(int c, int n, int per) {
    if (per) c = c < 0 ? c + n : (c >= n ? c - n : c);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// conductivity, 1/C and g = Tn + tau f/C of cell a
template <bool kSH>
__device__ __forceinline__ void cell_coef(const DevPhases& ph, double eps, double tau, const CoefIn& in, int64_t a,
                                          double& L, double& r, double& gv) {
    double t = in.T[a], a2 = in.alpha2[a];
    L = phys::cell_lambda<kSH>(ph, t, a2, in.m1, in.m2, a);
    r = inv_heat_capacity(ph, eps, t, a2, in.m1[a], in.m2[a]);
    double f = 0.0;
    if (in.src1) f += (1.0 - a2) * in.src1[a];
    if (in.src2) f += a2 * in.src2[a];
    gv = in.Tn[a] + tau * r * f;
}

template <bool kSH>
__global__ void __launch_bounds__(256) k_heat_coeffs_bound(DevGrid g, DevPhases ph, double eps, double tau, int face,
                                                           CoefIn in, double* __restrict__ Lam,
                                                           double* __restrict__ rC, double* __restrict__ rhs,
                                                           float* __restrict__ Lam32, float* __restrict__ rC32,
                                                           float* __restrict__ q32, float* __restrict__ w0,
                                                           double* __restrict__ lam) {
    // in-plane tile with halo: rows j0-1 .. j0+TY, columns i0-1 .. i0+TX
    __shared__ double sL[TY + 2][TX + 2], sG[TY + 2][TX + 2];
    __shared__ double zL[2][TY][TX], zG[2][TY][TX];  // layers k-1 and k+1
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY, k = blockIdx.z;
    const bool q = q32 != nullptr;
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
    const int kf = k;
    auto at = [&](int i, int j, int kk) {
        return (int64_t)fold_coord(i, g.nx, g.per[0]) + sy * fold_coord(j, g.ny, g.per[1]) +
               sz * fold_coord(kk, g.nz, g.per[2]);
    };
    // own cell (folded position)
    double L, r, gv;
    const int64_t a_self = at(i0 + tx, j0 + ty, kf);
    cell_coef<kSH>(ph, eps, tau, in, a_self, L, r, gv);
    sL[ty + 1][tx + 1] = L;
    sG[ty + 1][tx + 1] = gv;
    // halo: x sides (2 x TY cells), y sides (2 x TX cells), z layers (2 x TX x TY)
    if (tid < 2 * TY) {
        int side = tid / TY, jj = tid % TY;
        int ii = side ? i0 + TX : i0 - 1;
        double hl, hr, hg;
        cell_coef<kSH>(ph, eps, tau, in, at(ii, j0 + jj, kf), hl, hr, hg);
        sL[jj + 1][side ? TX + 1 : 0] = hl;
        sG[jj + 1][side ? TX + 1 : 0] = hg;
    }
    if (tid < 2 * TX) {
        int side = tid / TX, ii = tid % TX;
        int jj = side ? j0 + TY : j0 - 1;
        double hl, hr, hg;
        cell_coef<kSH>(ph, eps, tau, in, at(i0 + ii, jj, kf), hl, hr, hg);
        sL[side ? TY + 1 : 0][ii + 1] = hl;
        sG[side ? TY + 1 : 0][ii + 1] = hg;
    }
    if (g.nz > 1) {
        for (int side = 0; side < 2; ++side) {
            double hl, hr, hg;
            cell_coef<kSH>(ph, eps, tau, in, at(i0 + tx, j0 + ty, side ? k + 1 : k - 1), hl, hr, hg);
            zL[side][ty][tx] = hl;
            zG[side][ty][tx] = hg;
        }
    }
    __syncthreads();

    const int i = i0 + tx, j = j0 + ty;
    double bound = 0.0;
    if (i < g.nx && j < g.ny) {
        const int64_t a = a_self;
        Lam[a] = L;
        rC[a] = r;
        rhs[a] = gv;
        if (Lam32) {
            Lam32[a] = (float)L;
            rC32[a] = (float)r;
        }
        Faces fc;
        faces_of(g, i, j, k, fc);
        const double nbL[6] = {sL[ty + 1][tx], sL[ty + 1][tx + 2], sL[ty][tx + 1], sL[ty + 2][tx + 1],
                               g.nz > 1 ? zL[0][ty][tx] : 0.0, g.nz > 1 ? zL[1][ty][tx] : 0.0};
        double d = 0.0;
#pragma unroll
        for (int qf = 0; qf < 6; ++qf)
            if (fc.has[qf]) d += g.w[qf >> 1] * face_mean<double>(L, nbL[qf], face);
        bound = 2.0 * d * r;
        if (q) {
            const double nbG[6] = {sG[ty + 1][tx], sG[ty + 1][tx + 2], sG[ty][tx + 1], sG[ty + 2][tx + 1],
                                   g.nz > 1 ? zG[0][ty][tx] : 0.0, g.nz > 1 ? zG[1][ty][tx] : 0.0};
            const double Lf = (double)(float)L, rf = (double)(float)r;
            double S = 0.0;
#pragma unroll
            for (int qf = 0; qf < 6; ++qf)
                if (fc.has[qf]) S += g.w[qf >> 1] * face_mean<double>(Lf, (double)(float)nbL[qf], face) * (gv - nbG[qf]);
            q32[a] = (float)(-tau * rf * S);
            w0[a] = (float)(in.Tn[a] - gv);
        }
    }
    __shared__ double red[4];
    bound = wave_max(bound);
    if ((tid & 63) == 0) red[tid >> 6] = bound;
    __syncthreads();
    if (tid == 0) atomic_max_nonneg(lam + block_slot(), fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

template <bool kSH>
__global__ void __launch_bounds__(256) k_heat_coeffs(DevGrid g, DevPhases ph, double eps, double tau,
                                                     const double* __restrict__ T, const double* __restrict__ alpha2,
                                                     const double* __restrict__ m1, const double* __restrict__ m2,
                                                     const double* __restrict__ Tn, const double* __restrict__ src1,
                                                     const double* __restrict__ src2, double* __restrict__ Lam,
                                                     double* __restrict__ rC, double* __restrict__ rhs,
                                                     float* __restrict__ Lam32, float* __restrict__ rC32) {
    double B1 = ph.pinf[0] - ph.pinf[1];
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double t = T[a], a2 = alpha2[a], a1 = 1.0 - a2;
        double L = phys::cell_lambda<kSH>(ph, t, a2, m1, m2, a);
        double C1 = m1[a] * ph.cv[0], C2 = m2[a] * ph.cv[1];
        double C = C1 + C2;
        if (B1 != 0.0 && is_mixed(a2, eps)) C += B1 * B1 / (t * t * pressure_stiffness(ph, a2, C1, C2));
        double r = 1.0 / C;
        double f = 0.0;
        if (src1) f += a1 * src1[a];
        if (src2) f += a2 * src2[a];
        Lam[a] = L;
        if (rC) rC[a] = r;
        if (rhs) rhs[a] = Tn[a] + tau * r * f;
        if (Lam32) {
            Lam32[a] = (float)L;
            rC32[a] = (float)r;
        }
    }
}

__global__ void __launch_bounds__(256) k_visc_coeffs(DevGrid g, DevPhases ph, const double* __restrict__ alpha2,
                                                     const double* __restrict__ m1, const double* __restrict__ m2,
                                                     double* __restrict__ Lam, double* __restrict__ rC,
                                                     float* __restrict__ Lam32, float* __restrict__ rC32) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double a2 = alpha2[a];
        double mu = (1.0 - a2) * ph.mu[0] + a2 * ph.mu[1];
        double r = 1.0 / (m1[a] + m2[a]);
        Lam[a] = mu;
        rC[a] = r;
        if (Lam32) {
            Lam32[a] = (float)mu;
            rC32[a] = (float)r;
        }
    }
}

// --------------------------------------------------------------- reductions

// The Gershgorin bounds 2 rC sum_f w_f mean(Lambda_a, Lambda_b) of the three
// velocity components from one read of Lambda and 1/C: per cell the face
// means once, then each component's weighted sum (faces -x, +x, -y, +y, -z,
// +z) and its block max.
struct ViscW {
    double w[3][3];
};
__global__ void __launch_bounds__(256) k_gershgorin_visc(DevGrid g, int face, const double* __restrict__ Lam,
                                                         const double* __restrict__ rC, ViscW wc, int mask,
                                                         double* rows) {
    __shared__ double sh[16];
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    double mx[3] = {0.0, 0.0, 0.0};
    if (i < g.nx && j < g.ny) {
        int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        Faces f;
        faces_of(g, i, j, k, f);
        const double La = Lam[a], rc = rC[a];
        double m[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) m[q] = f.has[q] ? face_mean<double>(La, Lam[a + f.off[q]], face) : 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double d = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                if (f.has[q]) d += wc.w[c][q >> 1] * m[q];
            mx[c] = 2.0 * d * rc;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!((mask >> c) & 1)) continue;  // uniform
        const double b = block_max(mx[c], sh);
        if (flat_tid() == 0) atomic_max_nonneg(rows + (size_t)c * kSlots + block_slot(), b);
    }
}

__global__ void __launch_bounds__(256) k_energy(DevGrid g, DevPhases ph, const double* __restrict__ alpha2,
                                                const double* __restrict__ m1, const double* __restrict__ m2,
                                                const double* __restrict__ T1, const double* __restrict__ T2,
                                                double* energy) {
    __shared__ double sh[16];
    double e = 0.0;
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double a2 = alpha2[a];
        e += m1[a] * ph.cv[0] * T1[a] + m2[a] * ph.cv[1] * T2[a] + (1.0 - a2) * ph.pinf[0] + a2 * ph.pinf[1];
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) atomicAdd(energy + block_slot(), e);
}

__global__ void __launch_bounds__(256) k_pass_update(DevGrid g, DevPhases ph, double eps,
                                                     const double* __restrict__ Tit, const double* __restrict__ Tnew,
                                                     const double* __restrict__ Tn, const double* __restrict__ alpha2n,
                                                     const double* alpha2it, const double* __restrict__ m1,
                                                     const double* __restrict__ m2, double* alpha2out,
                                                     PassSlots ps) {
    double B1 = ph.pinf[0] - ph.pinf[1];
    PassAcc acc;
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double tn = Tnew[a], ti = Tit[a];
        acc.add(tn, ti);
        // d alpha2 = -B1/(T^2 W) dT from the step start, coefficient lagged at (T^(it), alpha2^(it))
        if (B1 != 0.0 && is_mixed(alpha2n[a], eps)) {
            double C1 = m1[a] * ph.cv[0], C2 = m2[a] * ph.cv[1];
            double W = pressure_stiffness(ph, alpha2it[a], C1, C2);
            alpha2out[a] = alpha2n[a] - B1 / (ti * ti * W) * (tn - Tn[a]);
        }
    }
    acc.store(ps);
}

__global__ void __launch_bounds__(256) k_be_residual(DevGrid g, int face, const double* __restrict__ v,
                                                     const double* __restrict__ rhs, const double* __restrict__ Lam,
                                                     const double* __restrict__ rC, double tau, double* rrp,
                                                     double* ggp) {
    __shared__ double sh[16];
    double rr = 0.0, gg = 0.0;
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_ijk(g, a, i, j, k);
        Faces f;
        faces_of(g, i, j, k, f);
        double S = stencil<double, double, double>(g, f, a, v, Lam, face);
        double C = 1.0 / rC[a];
        double r = C * (rhs[a] - v[a]) - tau * S;
        rr += r * r;
        gg += (C * rhs[a]) * (C * rhs[a]);
    }
    double s0 = block_sum(rr, sh);
    double s1 = block_sum(gg, sh);
    if (threadIdx.x == 0) {
        atomicAdd(rrp + block_slot(), s0);
        atomicAdd(ggp + block_slot(), s1);
    }
}

// ------------------------------------------------------------ LIM stages

// tau*b of a stage; with the bound on the device every wave folds its row
// (call before any lane leaves).
__device__ __forceinline__ double stage_tb(const StageParam& sp, double tau) {
    return sp.lam ? tau * row_max(sp.lam) * sp.chat : sp.tb;
}

__global__ void __launch_bounds__(256) k_stage64(DevGrid g, int face, const double* __restrict__ v,
                                                 const double* __restrict__ rhs, const double* __restrict__ Lam,
                                                 const double* __restrict__ rC, double* __restrict__ out,
                                                 StageParam sp, double tau) {
    const double tb = stage_tb(sp, tau), cm = 1.0 / (1.0 + tb);
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    Faces f;
    faces_of(g, i, j, k, f);
    double S = stencil<double, double, double>(g, f, a, v, Lam, face);
    out[a] = cm * (rhs[a] + tb * v[a] - tau * rC[a] * S);
}

__global__ void __launch_bounds__(256) k_final64(DevGrid g, int face, const double* __restrict__ v,
                                                 const double* __restrict__ rhs, const double* __restrict__ Lam,
                                                 const double* __restrict__ rC, double* __restrict__ out,
                                                 double tau, const double* __restrict__ Tit, PassSlots ps) {
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    PassAcc acc;
    if (i < g.nx && j < g.ny) {
        int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        Faces f;
        faces_of(g, i, j, k, f);
        // The flux w Lam_f (v_b - v_a) of a face is the same number with opposite
        // sign when evaluated from its other cell, so sum_a C_a (out_a - rhs_a)
        // cancels face by face (eq. LIM_last in conservative form).
        double S = stencil<double, double, double>(g, f, a, v, Lam, face);
        double t = rhs[a] - tau * rC[a] * S;
        out[a] = t;
        if (Tit) acc.add(t, Tit[a]);
    }
    if (Tit) acc.store(ps);
}

__global__ void __launch_bounds__(256) k_q32(DevGrid g, int face, const double* __restrict__ rhs,
                                             const double* __restrict__ v0, const float* __restrict__ Lam32,
                                             const float* __restrict__ rC32, double tau, float* __restrict__ q,
                                             float* __restrict__ w0) {
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    Faces f;
    faces_of(g, i, j, k, f);
    double S = stencil<double, double, float>(g, f, a, rhs, Lam32, face);
    q[a] = (float)(-tau * (double)rC32[a] * S);
    if (w0) w0[a] = (float)(v0[a] - rhs[a]);  // (not needed where v0 is rhs: w0 = 0)
}

__global__ void __launch_bounds__(256) k_stage32(DevGrid g, int face, const float* __restrict__ w,
                                                 const float* __restrict__ q, const float* __restrict__ Lam32,
                                                 const float* __restrict__ rC32, float* __restrict__ out,
                                                 StageParam sp, double tau) {
    const double tbd = stage_tb(sp, tau);
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    const float tb = (float)tbd, cm = (float)(1.0 / (1.0 + tbd)), tf = (float)tau;
    Faces f;
    faces_of(g, i, j, k, f);
    float S = stencil<float, float, float>(g, f, a, w, Lam32, face);
    out[a] = cm * (q[a] + tb * w[a] - tf * rC32[a] * S);
}

__global__ void __launch_bounds__(256) k_final32(DevGrid g, int face, const float* __restrict__ w,
                                                 const double* __restrict__ rhs, const float* __restrict__ Lam32,
                                                 const double* __restrict__ rC, double* __restrict__ out,
                                                 double tau, const double* __restrict__ Tit, PassSlots ps) {
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    PassAcc acc;
    if (i < g.nx && j < g.ny) {
        int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        Faces f;
        faces_of(g, i, j, k, f);
        double va = rhs[a] + (double)w[a], La = (double)Lam32[a], S = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (!f.has[q]) continue;
            int64_t b = a + f.off[q];
            S += g.w[q >> 1] * face_mean<double>(La, (double)Lam32[b], face) * (va - (rhs[b] + (double)w[b]));
        }
        double t = rhs[a] - tau * rC[a] * S;
        out[a] = t;
        if (Tit) acc.add(t, Tit[a]);
    }
    if (Tit) acc.store(ps);
}

// ----------------------------------------------------------------- adjoint

__global__ void __launch_bounds__(256) k_adj_stage(DevGrid g, int face, const double* __restrict__ lam,
                                                   const double* __restrict__ vprev, const double* __restrict__ Lam,
                                                   const double* __restrict__ rC, double* __restrict__ lam_out,
                                                   double* __restrict__ dg, double* __restrict__ gLam, double cm,
                                                   double tb, double tau) {
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    Faces f;
    faces_of(g, i, j, k, f);
    double la = lam[a] * rC[a], La = Lam[a], va = vprev[a];
    double Sadj = 0.0, G = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!f.has[q]) continue;
        int64_t b = a + f.off[q];
        double Lb = Lam[b], lb = lam[b] * rC[b], w = g.w[q >> 1];
        Sadj += w * face_mean<double>(La, Lb, face) * (lb - la);
        G += cm * tau * w * (vprev[b] - va) * (la - lb) * face_partial<double>(La, Lb, face);
    }
    dg[a] += cm * lam[a];
    gLam[a] += G;
    lam_out[a] = cm * (tb * lam[a] + tau * Sadj);
}

__global__ void __launch_bounds__(256) k_adj_cell(DevGrid g, DevPhases ph, const double* __restrict__ Tit,
                                                  const double* __restrict__ alpha2, const double* __restrict__ m1,
                                                  const double* __restrict__ m2, const double* __restrict__ gLam,
                                                  const double* __restrict__ dg, const double* __restrict__ lam0,
                                                  double* __restrict__ acc, double* __restrict__ mu, int first_pass,
                                                  const double* __restrict__ rCpsi, double* k0a, double* k0b,
                                                  int init) {
    __shared__ double sh[16];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N;
         a += (int64_t)gridDim.x * blockDim.x) {
        double t = Tit[a], a2 = alpha2[a], gl = gLam[a];
        // lambda form, or psi = C^-1 lambda form (rCpsi = 1/C): lambda = psi / rC
        const double acc0 = init ? 0.0 : acc[a];
        double acc_a = rCpsi ? acc0 + (dg[a] + lam0[a]) / rCpsi[a] : acc0 + dg[a] + lam0[a];
        double dk[2], dL;
        phys::cell_conductivity_grad(ph, t, a2, phys::mix_density(ph, m1, m2, a), dk, dL);
        s0 += gl * dk[0];
        s1 += gl * dk[1];
        double m = gl * dL;
        mu[a] = m;
        acc[a] = first_pass ? acc_a + m : acc_a;
    }
    double r0 = block_sum(s0, sh);
    double r1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        atomicAdd(k0a + block_slot(), r0);
        atomicAdd(k0b + block_slot(), r1);
    }
}

__global__ void __launch_bounds__(256) k_visc_heat(DevGrid g, DevPhases ph, double eps, int face, double tau,
                                                   const double* __restrict__ alpha2, const double* __restrict__ m1,
                                                   const double* __restrict__ m2, const double* __restrict__ mu,
                                                   const double* __restrict__ uh64, const double* __restrict__ g64,
                                                   const float* __restrict__ w32, double* T1, double* T2,
                                                   double* E) {
    int i = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const int64_t a = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    auto uh = [&](int64_t c) { return uh64 ? uh64[c] : g64[c] + (double)w32[c]; };
    Faces f;
    faces_of(g, i, j, k, f);
    const double ua = uh(a), a2a = alpha2[a], mua = mu[a];
    double e1 = 0.0, e2 = 0.0, work = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!f.has[q]) continue;
        const int64_t b = a + f.off[q];
        const double ub = uh(b);
        const double du = ub - ua;
        const double wmu = g.w[q >> 1] * face_mean<double>(mua, mu[b], face);
        // total energy: uh_f times the flux w mu_f (uh_b - uh_a) through the face
        work += 0.5 * (ua + ub) * wmu * du;
        const double d = 0.5 * wmu * du * du;
        const double a2f = 0.5 * (a2a + alpha2[b]);
        e1 += (1.0 - a2f) * d;
        e2 += a2f * d;
    }
    if (E) E[a] += tau * work;
    if (!T1) return;
    e1 *= tau;
    e2 *= tau;
    const double C1 = m1[a] * ph.cv[0], C2 = m2[a] * ph.cv[1];
    if (a2a <= eps) {
        T1[a] += (e1 + e2) / C1;
    } else if (a2a >= 1.0 - eps) {
        T2[a] += (e1 + e2) / C2;
    } else {
        T1[a] += e1 / C1;
        T2[a] += e2 / C2;
    }
}

// Total energy of the heat part: the last pass's final stage moved
// C_eff (T^{n+1} - T^n) into each cell.
__global__ void __launch_bounds__(256) k_total_energy_heat(int64_t n, const double* __restrict__ T,
                                                           const double* __restrict__ Tn,
                                                           const double* __restrict__ rC, double* __restrict__ E) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x)
        E[a] += (T[a] - Tn[a]) / rC[a];
}

// One wave per target row folds its kSlots slots with the target's
// operation; consume = 1 also clears the row for its next use.  With
// move_from >= 0 the wave of row t0 then moves row move_from into it (and
// clears move_from): each lane touches only its own slots, in order.
__global__ void __launch_bounds__(64) k_collect(double* __restrict__ acc, PassResult* res, int t0, int consume,
                                                int move_from, unsigned long long seq, unsigned* done) {
    const int t = t0 + blockIdx.x, lane = threadIdx.x;
    double* row = acc + (int64_t)t * kSlots;
    const bool sum = tgt_is_sum(t);
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kSlots / 64; ++k) v = sum ? v + row[lane + 64 * k] : fmax(v, row[lane + 64 * k]);
    if (consume) {
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) row[lane + 64 * k] = 0.0;
    }
    if (move_from >= 0 && blockIdx.x == 0) {
        double* f = acc + (int64_t)move_from * kSlots;
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) {
            row[lane + 64 * k] = f[lane + 64 * k];
            f[lane + 64 * k] = 0.0;
        }
    }
    v = sum ? wave_sum(v) : wave_max(v);
    if (lane == 0) {
        res->v[t] = v;
        if (seq) {
            // each workgroup releases its value to the host before it counts
            // itself in; the last one publishes seq after all of them
            __threadfence_system();
            const unsigned n = __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (n == gridDim.x - 1) {
                __threadfence_system();
                __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&res->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_fill(double* p, double v, int64_t n) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x)
        p[a] = v;
}

__global__ void __launch_bounds__(256) k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x)
        d[a] = s[a];
}

// Field copies between the caller's precision and the state's float64.
template <typename To, typename From>
__global__ void __launch_bounds__(256) k_convert(To* __restrict__ d, const From* __restrict__ s, int64_t n) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x)
        d[a] = (To)s[a];
}

}  // namespace

// ------------------------------------------------------------------ launches

namespace {
// Grid-stride launches use enough blocks to keep every CU busy.
int pointwise_blocks(int64_t N) {
    int64_t b = (N + kReduceThreads - 1) / kReduceThreads;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}
}  // namespace

void launch_zero_rows(hipStream_t s, double* acc, int t0, int t1) {
    int64_t n = (int64_t)(t1 - t0) * kSlots;
    hipLaunchKernelGGL(k_fill, dim3(pointwise_blocks(n)), dim3(256), 0, s, acc + (int64_t)t0 * kSlots, 0.0, n);
}

void launch_collect(hipStream_t s, double* acc, PassResult* res, int t0, int t1, int consume, int move_from,
                    unsigned long long seq, unsigned* done) {
    hipLaunchKernelGGL(k_collect, dim3(t1 - t0), dim3(64), 0, s, acc, res, t0, consume, move_from, done ? seq : 0ULL,
                       done);
}

void launch_relax(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double* alpha2,
                  const double* m1, const double* m2, double* T1, double* T2, double* Tn, double* a2n) {
    hipLaunchKernelGGL(k_relax, dim3(pointwise_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, eps, alpha2, m1, m2,
                       T1, T2, Tn, a2n);
}

void launch_heat_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau,
                        const double* T, const double* alpha2, const double* m1, const double* m2,
                        const double* Tn, const double* src1, const double* src2, double* Lam, double* rC,
                        double* rhs, float* Lam32, float* rC32) {
    if (ph.spitzer)
        hipLaunchKernelGGL(k_heat_coeffs<true>, dim3(pointwise_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, eps,
                           tau, T, alpha2, m1, m2, Tn, src1, src2, Lam, rC, rhs, Lam32, rC32);
    else
        hipLaunchKernelGGL(k_heat_coeffs<false>, dim3(pointwise_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, eps,
                           tau, T, alpha2, m1, m2, Tn, src1, src2, Lam, rC, rhs, Lam32, rC32);
}

void launch_heat_coeffs_bound(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                              const double* T, const double* alpha2, const double* m1, const double* m2,
                              const double* Tn, const double* src1, const double* src2, double* Lam, double* rC,
                              double* rhs, float* Lam32, float* rC32, float* q32, float* w0, double* lam) {
    CoefIn in{T, alpha2, m1, m2, Tn, src1, src2};
    if (ph.spitzer)
        hipLaunchKernelGGL(k_heat_coeffs_bound<true>, tile_grid(g), dim3(TX, TY), 0, s, g, ph, eps, tau, face, in, Lam,
                           rC, rhs, Lam32, rC32, q32, w0, lam);
    else
        hipLaunchKernelGGL(k_heat_coeffs_bound<false>, tile_grid(g), dim3(TX, TY), 0, s, g, ph, eps, tau, face, in, Lam,
                           rC, rhs, Lam32, rC32, q32, w0, lam);
}

void launch_visc_coeffs(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2,
                        const double* m1, const double* m2, double* Lam, double* rC, float* Lam32, float* rC32) {
    hipLaunchKernelGGL(k_visc_coeffs, dim3(pointwise_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, alpha2, m1, m2,
                       Lam, rC, Lam32, rC32);
}

void launch_gershgorin_visc(hipStream_t s, const DevGrid& g, int face, const double* Lam, const double* rC,
                            const double wc[3][3], int mask, double* rows) {
    ViscW w;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) w.w[c][d] = wc[c][d];
    hipLaunchKernelGGL(k_gershgorin_visc, tile_grid(g), dim3(TX, TY), 0, s, g, face, Lam, rC, w, mask, rows);
}


void launch_energy(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* alpha2, const double* m1,
                   const double* m2, const double* T1, const double* T2, double* energy) {
    hipLaunchKernelGGL(k_energy, dim3(reduce_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, alpha2, m1, m2, T1, T2,
                       energy);
}

void launch_stage64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, StageParam sp, double tau) {
    hipLaunchKernelGGL(k_stage64, tile_grid(g), dim3(TX, TY), 0, s, g, face, v, rhs, Lam, rC, out, sp, tau);
}

void launch_final64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, double tau, const double* Tit, PassSlots ps) {
    hipLaunchKernelGGL(k_final64, tile_grid(g), dim3(TX, TY), 0, s, g, face, v, rhs, Lam, rC, out, tau, Tit, ps);
}

void launch_q32(hipStream_t s, const DevGrid& g, int face, const double* rhs, const double* v0,
                const float* Lam32, const float* rC32, double tau, float* q, float* w0) {
    hipLaunchKernelGGL(k_q32, tile_grid(g), dim3(TX, TY), 0, s, g, face, rhs, v0, Lam32, rC32, tau, q, w0);
}

void launch_stage32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* q,
                    const float* Lam32, const float* rC32, float* out, StageParam sp, double tau) {
    hipLaunchKernelGGL(k_stage32, tile_grid(g), dim3(TX, TY), 0, s, g, face, w, q, Lam32, rC32, out, sp, tau);
}

void launch_final32(hipStream_t s, const DevGrid& g, int face, const float* w, const double* rhs,
                    const float* Lam32, const double* rC, double* out, double tau, const double* Tit, PassSlots ps) {
    hipLaunchKernelGGL(k_final32, tile_grid(g), dim3(TX, TY), 0, s, g, face, w, rhs, Lam32, rC, out, tau, Tit, ps);
}

void launch_pass_update(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, const double* Tit,
                        const double* Tnew, const double* Tn, const double* alpha2n, const double* alpha2it,
                        const double* m1, const double* m2, double* alpha2out, PassSlots ps) {
    hipLaunchKernelGGL(k_pass_update, dim3(reduce_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, eps, Tit, Tnew,
                       Tn, alpha2n, alpha2it, m1, m2, alpha2out, ps);
}

void launch_be_residual(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                        const double* Lam, const double* rC, double tau, double* rr, double* gg) {
    hipLaunchKernelGGL(k_be_residual, dim3(reduce_blocks(g.N)), dim3(kReduceThreads), 0, s, g, face, v, rhs, Lam,
                       rC, tau, rr, gg);
}

void launch_adj_stage(hipStream_t s, const DevGrid& g, int face, const double* lam, const double* vprev,
                      const double* Lam, const double* rC, double* lam_out, double* dg, double* gLam, double cm,
                      double tb, double tau) {
    hipLaunchKernelGGL(k_adj_stage, tile_grid(g), dim3(TX, TY), 0, s, g, face, lam, vprev, Lam, rC, lam_out, dg,
                       gLam, cm, tb, tau);
}

void launch_adj_cell(hipStream_t s, const DevGrid& g, const DevPhases& ph, const double* Tit, const double* alpha2,
                     const double* m1, const double* m2, const double* gLam, const double* dg, const double* lam0,
                     double* acc, double* mu, int first_pass, const double* rCpsi, double* k0a, double* k0b,
                     int init) {
    hipLaunchKernelGGL(k_adj_cell, dim3(reduce_blocks(g.N)), dim3(kReduceThreads), 0, s, g, ph, Tit, alpha2, m1, m2,
                       gLam, dg, lam0, acc, mu, first_pass, rCpsi, k0a, k0b, init);
}

void launch_visc_heat(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, int face, double tau,
                      const double* alpha2, const double* m1, const double* m2, const double* mu,
                      const double* uh64, const double* g64, const float* w32, double* T1, double* T2,
                      double* E) {
    hipLaunchKernelGGL(k_visc_heat, tile_grid(g), dim3(TX, TY), 0, s, g, ph, eps, face, tau, alpha2, m1, m2, mu, uh64,
                       g64, w32, T1, T2, E);
}

void launch_total_energy_heat(hipStream_t s, int64_t N, const double* T, const double* Tn, const double* rC,
                              double* E) {
    hipLaunchKernelGGL(k_total_energy_heat, dim3(pointwise_blocks(N)), dim3(256), 0, s, N, T, Tn, rC, E);
}

void launch_fill(hipStream_t s, double* p, double v, int64_t n) {
    hipLaunchKernelGGL(k_fill, dim3(pointwise_blocks(n)), dim3(256), 0, s, p, v, n);
}

void launch_copy(hipStream_t s, double* dst, const double* src, int64_t n) {
    hipLaunchKernelGGL(k_copy, dim3(pointwise_blocks(n)), dim3(256), 0, s, dst, src, n);
}

void launch_widen(hipStream_t s, double* dst, const float* src, int64_t n) {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(pointwise_blocks(n)), dim3(256), 0, s, dst, src, n);
}

void launch_narrow(hipStream_t s, float* dst, const double* src, int64_t n) {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(pointwise_blocks(n)), dim3(256), 0, s, dst, src, n);
}

}  // namespace tlim
