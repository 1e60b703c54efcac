// One heat step of a 2D grid in a single cooperative launch (Sec. 3.4:
// temperature relaxation, then Algorithm 1's Picard passes of eq. LIM with
// the final stage eq. LIM_last), for grids whose tiles all fit on the chip
// at once (a 1024^2 grid in FP64 takes 250 of the 256 CUs).
//
// Every workgroup owns one 64 x 128 extended tile for the whole step (16
// wave64s of 8 rows, one column per lane, as the blocked sweep kernel) and
// keeps its state on chip: the stage iterate v and the four face
// coefficients kappa in registers, g = T^n in LDS.  Between the steps of the
// method the workgroups meet at grid barriers:
//   1. relax every cell of the tile, build Lambda, 1/C and kappa, and the
//      bound lambda_G of the output cells (max into the pass row); barrier;
//   2. per Picard pass: fold lambda_G, P = ceil(pi/4 sqrt(tau lambda_G + 1))
//      and the stage parameters b_m = lambda_G chat_m of that P (table from
//      the host), then the 2P-1 stages in blocks of at most H: a block leaves
//      the output cells (H in from the tile edge) exact; between blocks the
//      output cells go to an exchange array, barrier, and the ring of H cells
//      around them is read back from the neighbours' output cells;
//   3. at the end of a pass: the Picard reductions, T^(it+1) of the output
//      cells and the next pass's bound there (the last block of a pass that
//      is followed by another has at most H-1 stages, so T^(it+1) is exact
//      one cell beyond the output cells); barrier; the ring of T^(it+1) read
//      back and the next pass's kappa; v restarts from g.
// All workgroups take the same branches (P comes from the same reduced
// lambda_G), so every one reaches every barrier.  The barrier waits are
// bounded: a workgroup that waits too long adds 1 to the flag row and goes
// on; the host then treats the step as lost (alpha2, T1 and T2 must be set again).
// Data one workgroup writes and another reads within the launch (relaxed
// alpha2, 1/C, the exchange arrays, the pass results, the reduction rows)
// moves by device-coherent loads and stores, so a barrier needs no cache
// write-back or invalidation: each wave waits for its stores, then one
// thread per workgroup counts in and polls.
#include <hip/hip_runtime.h>

#include "tlim_device.h"
#include "tlim_internal.h"

namespace tlim {

namespace {

using phys::cell_conductivity;
using phys::inv_heat_capacity;
using phys::relax_cell;
using tb::fmean;
using tb::fold;
using tb::from_left;
using tb::from_right;
using tb::lane_value;
using tb::ROWS;
using tb::row_index;

constexpr int NW = 16;          // waves per workgroup
constexpr int EY = NW * ROWS;   // rows of the extended tile
constexpr int kHmin = 4, kHmax = 12;
constexpr double kPiQuarter = 3.14159265358979323846 / 4.0;

struct StepArgs {
    DevPhases ph;
    double eps, tau;
    Step2D st;
    int face, nx, ny, perx, pery;
    double wx, wy;
    int H, tiles_x, ox, oy;
};

// Device-coherent access to data shared between workgroups in the launch.
__device__ __forceinline__ void cstore(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double cload(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Opaque copy of an integer: keeps the compiler from hoisting index
// arithmetic out of the pass loop (which would hold it in registers across
// the stage loop).
__device__ __forceinline__ int fresh(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Barrier over all workgroups of the launch (all resident).  Workgroup b
// stores the barrier's number g into its own arrival word bar[b]; the first
// wave of every workgroup then polls all arrival words until each holds at
// least g.  No word is written by more than one workgroup, so arrivals do not
// queue on one address.
__device__ void grid_barrier(unsigned* bar, unsigned g, double* flag, unsigned limit) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's coherent stores have landed
    __syncthreads();
    const unsigned nblk = gridDim.x;
    if (threadIdx.x == 0) __hip_atomic_store(bar + blockIdx.x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < 64) {
        const unsigned lane = threadIdx.x;
        unsigned spins = 0;
        for (;;) {
            // the arrival words in batches of 4 per lane, each batch in
            // flight at once (a resident grid fits one batch)
            bool here = true;
            for (unsigned b0 = 0; b0 < nblk; b0 += 256) {
                unsigned w[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const unsigned b = b0 + lane + 64u * k;
                    w[k] = b < nblk ? __hip_atomic_load(bar + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : g;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) here = here && w[k] >= g;
            }
            if (__all(here)) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > limit) {
                if (lane == 0) atomicAdd(flag, 1.0);
                break;
            }
        }
    }
    __syncthreads();
}

// Lambda of a cell under the law family the kernel is compiled for (kSH: a
// phase follows the Spitzer-Harm law, which needs rho = m1 + m2; the power
// law ignores rho).
template <bool kSH>
__device__ __forceinline__ double step_lambda(const StepArgs& a, double t, double a2, double rho) {
    if constexpr (kSH) return cell_conductivity(a.ph, t, a2, rho);
    else return phys::cell_conductivity_pow(a.ph, t, a2);
}

template <bool kSH>
__global__ void __launch_bounds__(64 * NW, 4) k_step2d(StepArgs a) {
    __shared__ double sG[EY][64];
    __shared__ double sh_lo[2][NW][64], sh_hi[2][NW][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int H = a.H;
    const int tile = tb::xcd_block();  // tiles in XCD order (neighbours share an L2)
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const int xg = tx * a.ox - H + lane;
    const int yg0 = ty * a.oy - H + wv * ROWS;
    const int xi = fold(xg, a.nx, a.perx);
    const int yi0 = fold(yg0, a.ny, a.pery);
    const bool inx = xg >= 0 && xg < a.nx;
    const bool fL = a.perx ? a.nx > 1 : (inx && xg > 0);
    const bool fR = a.perx ? a.nx > 1 : (inx && xg < a.nx - 1);
    const bool xout = lane >= H && lane < 64 - H && xg < a.nx;
    const int wdn = wv > 0 ? wv - 1 : 0, wup = wv < NW - 1 ? wv + 1 : wv;
    const int slot = (int)(((int64_t)blockIdx.x * NW + wv) % kSlots);
    double* const flag = a.st.acc + (size_t)kTgtFlag * kSlots;
    unsigned nbar = 0;
    int sb = 0;  // seam buffer of the next exchange (alternates)

    // bit r: row r of this lane is an output cell of the tile
    unsigned outmask = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int row = wv * ROWS + r;
        if (xout && row >= H && row < EY - H && yg0 + r < a.ny) outmask |= 1u << r;
    }
    auto out_cell = [&](int r) { return ((outmask >> r) & 1u) != 0; };
    // element offsets (the launcher requires N < 2^31)
    auto cell_idx = [&](int r) { return row_index(fresh(yi0), yg0, r, a.ny, a.pery) * a.nx + fresh(xi); };
    auto out_idx = [&](int r) { return (fresh(yg0) + r) * a.nx + fresh(xg); };
    auto face_d = [&](int r) {
        const int y = yg0 + r;
        return a.pery ? a.ny > 1 : (y >= 0 && y < a.ny && y > 0);
    };
    auto face_u = [&](int r) {
        const int y = yg0 + r;
        return a.pery ? a.ny > 1 : (y >= 0 && y < a.ny && y < a.ny - 1);
    };

    double v[ROWS], kL[ROWS], kR[ROWS], kD[ROWS], kU[ROWS];

    // Face coefficients kappa = tau rC w Lambda_f of every cell from the cell
    // conductivities L (y seams through LDS), and the Gershgorin bound
    // 2 rC sum_f w Lambda_f of the output cells (faces -x, +x, -y, +y) into
    // slot `slot` of row `lam_row`.
    auto build = [&](const double* L, const double* rc, double* lam_row, bool kappa) {
        sh_lo[sb][wv][lane] = L[0];
        sh_hi[sb][wv][lane] = L[ROWS - 1];
        __syncthreads();
        const double sdn = sh_hi[sb][wdn][lane], sup = sh_lo[sb][wup][lane];
        sb ^= 1;
        const double Ldn = wv > 0 ? sdn : L[0];
        const double Lup = wv < NW - 1 ? sup : L[ROWS - 1];
        double bound = 0.0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const bool fD = face_d(r), fU = face_u(r);
            const double Ll = from_left(L[r]), Lr = from_right(L[r]);
            const double Ld = r > 0 ? L[r - 1] : Ldn;
            const double Lu = r < ROWS - 1 ? L[r + 1] : Lup;
            if (kappa) {
                const double t = a.tau * rc[r];
                kL[r] = fL ? t * a.wx * fmean<double>(L[r], Ll, a.face) : 0.0;
                kR[r] = fR ? t * a.wx * fmean<double>(L[r], Lr, a.face) : 0.0;
                kD[r] = fD ? t * a.wy * fmean<double>(L[r], Ld, a.face) : 0.0;
                kU[r] = fU ? t * a.wy * fmean<double>(L[r], Lu, a.face) : 0.0;
            }
            if (lam_row && out_cell(r)) {
                double d = 0.0;
                if (fL) d += a.wx * fmean<double>(L[r], Ll, a.face);
                if (fR) d += a.wx * fmean<double>(L[r], Lr, a.face);
                if (fD) d += a.wy * fmean<double>(L[r], Ld, a.face);
                if (fU) d += a.wy * fmean<double>(L[r], Lu, a.face);
                bound = fmax(bound, 2.0 * d * rc[r]);
            }
        }
        if (lam_row) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
            if (lane == 0)
                atomicMax((unsigned long long*)(lam_row + slot),
                          (unsigned long long)__double_as_longlong(bound + 0.0));
        }
    };

    // ---- 1. relaxation and the first pass's coefficients
    {
        double L[ROWS], rc[ROWS];
        // the inputs of all rows in flight before the relaxation (T2 may alias T1)
        const double* const T2p = a.st.T2 ? a.st.T2 : a.st.T1;
        double t1[ROWS], t2[ROWS], m1[ROWS], m2[ROWS], a20[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int idx = cell_idx(r);
            t1[r] = a.st.T1[idx];
            t2[r] = T2p[idx];
            m1[r] = a.st.m1[idx];
            m2[r] = a.st.m2[idx];
            a20[r] = a.st.alpha2[idx];
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            double T, a2;
            relax_cell(a.ph, a.eps, a20[r], t1[r], t2[r], m1[r], m2[r], T, a2);
            rc[r] = inv_heat_capacity(a.ph, a.eps, T, a2, m1[r], m2[r]);
            L[r] = step_lambda<kSH>(a, T, a2, m1[r] + m2[r]);
            sG[wv * ROWS + r][lane] = T;
            if (out_cell(r)) {
                const int o = out_idx(r);
                a.st.Tn[o] = T;
                cstore(a.st.a2n + o, a2);
                cstore(a.st.rC + o, rc[r]);
            }
        }
        build(L, rc, a.st.acc + (size_t)tgt_lam(0) * kSlots, true);
    }
    grid_barrier(a.st.bar, ++nbar, flag, a.st.spin_limit);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) v[r] = sG[wv * ROWS + r][lane];

    int xb = 0;  // exchange array of the next block boundary
    for (int it = 0; it < a.st.passes; ++it) {
        // lambda_G of the pass and its schedule (the same in every workgroup)
        const double* lrow = a.st.acc + (size_t)tgt_lam(it) * kSlots;
        double lam = 0.0;
#pragma unroll
        for (int k = 0; k < kSlots / 64; ++k) lam = fmax(lam, cload(lrow + lane + 64 * k));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o, 64));
        const double z = __dadd_rn(__dmul_rn(a.tau, lam), 1.0);
        const double Pd = ceil(__dmul_rn(kPiQuarter, sqrt(z)));
        if (blockIdx.x == 0 && wv == 0) {
            double* prow = a.st.acc + (size_t)(kTgtP0 + it) * kSlots;
#pragma unroll
            for (int k = 0; k < kSlots / 64; ++k) prow[lane + 64 * k] = (lane == 0 && k == 0) ? Pd : 0.0;
        }
        if (!(Pd >= 1.0 && Pd <= (double)a.st.pmax)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(flag, 1.0);
            return;  // every workgroup leaves here, before any further barrier
        }
        const int P = (int)Pd;
        const int nst = 2 * P - 1;
        const double* chat = a.st.chat + (size_t)(P - 1) * (P - 1);
        // blocks of at most H stages; before another pass the last block has
        // at most H-1, so the new iterate is exact one cell beyond the output
        // cells and their bound needs no exchange
        int nblocks = (nst + H - 1) / H;
        int K0 = (nst + nblocks - 1) / nblocks;
        if (it + 1 < a.st.passes && nst - (nblocks - 1) * K0 > H - 1) {
            ++nblocks;
            K0 = (nst + nblocks - 1) / nblocks;
        }

        int m = 0;
        while (m < nst) {
            const int K = nst - m < K0 ? nst - m : K0;
            // lane q holds tau b and 1/(1 + tau b) of stage m + q
            double ptb = 0.0, pcm = 1.0;
            if (lane < K) {
                ptb = a.tau * lam * chat[m + lane];
                pcm = 1.0 / (1.0 + ptb);
            }
            for (int s = 0; s < K; ++s) {
                sh_lo[sb][wv][lane] = v[0];
                sh_hi[sb][wv][lane] = v[ROWS - 1];
                __syncthreads();
                const double sdn = sh_hi[sb][wdn][lane], sup = sh_lo[sb][wup][lane];
                sb ^= 1;
                const double vdn = wv > 0 ? sdn : v[0];
                const double vup = wv < NW - 1 ? sup : v[ROWS - 1];
                const double tb = lane_value(ptb, s), cm = lane_value(pcm, s);
                // face differences shared by the face's two cells (exact)
                double ddn = v[0] - vdn;
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const double c = v[r];
                    const double up = r < ROWS - 1 ? v[r + 1] : vup;
                    const double drt = c - from_right(c);
                    const double dlf = -from_left(drt);
                    const double dup = c - up;
                    const double S = kL[r] * dlf + kR[r] * drt + kD[r] * ddn + kU[r] * dup;
                    v[r] = cm * (sG[wv * ROWS + r][lane] + tb * c - S);
                    ddn = -dup;
                }
            }
            m += K;
            if (m < nst) {
                // block boundary: publish the exact output cells, read back the ring
                double* xa = a.st.vx[xb];
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    if (out_cell(r)) cstore(xa + out_idx(r), v[r]);
                grid_barrier(a.st.bar, ++nbar, flag, a.st.spin_limit);
                // every row's word in flight at once (an output cell reads
                // back what it published), then the ring keeps its values
                double w[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) w[r] = cload(xa + cell_idx(r));
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    if (!out_cell(r)) v[r] = w[r];
                xb ^= 1;
            }
        }

        // ---- 3. end of the pass: reductions and T^(it+1) of the output cells
        {
            double* Tw = a.st.Tout[it & 1];
            const double* Tprev = a.st.Tout[(it + 1) & 1];
            double dmax = 0.0, tmax = 0.0, bad = 0.0;
            double tp[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
                tp[r] = it == 0 ? sG[wv * ROWS + r][lane] : cload(Tprev + (out_cell(r) ? out_idx(r) : 0));
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                if (out_cell(r)) {
                    const int o = out_idx(r);
                    const double tn = v[r];
                    const double tit = tp[r];
                    dmax = fmax(dmax, fabs(tn - tit));
                    tmax = fmax(tmax, fabs(tn));
                    if (!(tn > 0.0) || isinf(tn)) bad += 1.0;
                    cstore(Tw + o, tn);
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
                tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
                bad += __shfl_xor(bad, o, 64);
            }
            if (lane == 0) {
                double* acc = a.st.acc;
                atomicMax((unsigned long long*)(acc + (size_t)tgt_dmax(it) * kSlots + slot),
                          (unsigned long long)__double_as_longlong(dmax + 0.0));
                atomicMax((unsigned long long*)(acc + (size_t)tgt_tmax(it) * kSlots + slot),
                          (unsigned long long)__double_as_longlong(tmax + 0.0));
                if (bad != 0.0) atomicAdd(acc + (size_t)tgt_bad(it) * kSlots + slot, bad);
            }
            if (it + 1 < a.st.passes) {
                // The next pass's bound from the cells this tile has exact (the
                // output cells and one ring), then its kappa on the whole tile
                // after the exchange.  alpha2 and 1/C were written before the
                // first barrier and not since: plain loads see them.
                double L[ROWS], rc[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const int idx = cell_idx(r);
                    L[r] = step_lambda<kSH>(a, v[r], a.st.a2n[idx], kSH ? a.st.m1[idx] + a.st.m2[idx] : 1.0);
                    rc[r] = a.st.rC[idx];
                }
                build(L, rc, a.st.acc + (size_t)tgt_lam(it + 1) * kSlots, false);
                grid_barrier(a.st.bar, ++nbar, flag, a.st.spin_limit);
                double w[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) w[r] = cload(Tw + cell_idx(r));
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    if (!out_cell(r)) {
                        const int idx = cell_idx(r);
                        L[r] = step_lambda<kSH>(a, w[r], a.st.a2n[idx], kSH ? a.st.m1[idx] + a.st.m2[idx] : 1.0);
                    }
                }
                build(L, rc, nullptr, true);
#pragma unroll
                for (int r = 0; r < ROWS; ++r) v[r] = sG[wv * ROWS + r][lane];
            }
        }
    }
}

struct Tiling {
    int H, tiles_x, tiles_y;
};

int resident_limit() {
    static int limit = -1;
    if (limit < 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step2d<true>, 64 * NW, 0) != hipSuccess)
            limit = 0;
        else
            limit = cus * per;
    }
    return limit;
}

// The widest ring H (fewest blocks per pass) whose tiling is resident.
Tiling tiling_of(const DevGrid& g) {
    Tiling t{0, 0, 0};
    if (g.nz != 1 || g.ny < EY || g.nx < 2 || g.N >= ((int64_t)1 << 31)) return t;
    const int limit = resident_limit();
    for (int H = kHmax; H >= kHmin; --H) {
        const int tx = (g.nx + 64 - 2 * H - 1) / (64 - 2 * H);
        const int ty = (g.ny + EY - 2 * H - 1) / (EY - 2 * H);
        if ((int64_t)tx * ty <= limit && tx * ty <= kStepMaxTiles) return Tiling{H, tx, ty};
    }
    return t;
}

}  // namespace

int step2d_tiles(const DevGrid& g) {
    const Tiling t = tiling_of(g);
    return t.H ? t.tiles_x * t.tiles_y : 0;
}

bool launch_step2d(hipStream_t s, const DevGrid& g, const DevPhases& ph, double eps, double tau, int face,
                   const Step2D& st) {
    const Tiling t = tiling_of(g);
    if (!t.H) return false;
    StepArgs a{};
    a.ph = ph;
    a.eps = eps;
    a.tau = tau;
    a.st = st;
    a.face = face;
    a.nx = g.nx;
    a.ny = g.ny;
    a.perx = g.per[0];
    a.pery = g.per[1];
    a.wx = g.w[0];
    a.wy = g.w[1];
    a.H = t.H;
    a.tiles_x = t.tiles_x;
    a.ox = 64 - 2 * t.H;
    a.oy = EY - 2 * t.H;
    void* args[] = {&a};
    const void* kern = ph.spitzer ? (const void*)k_step2d<true> : (const void*)k_step2d<false>;
    const hipError_t e = hipLaunchCooperativeKernel(kern, dim3((unsigned)(t.tiles_x * t.tiles_y)),
                                                    dim3(64 * NW), args, 0, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

}  // namespace tlim
