// The Gershgorin bound of the heat operator without a context or any device
// allocation (tlim_spectral_bound_noalloc): for callers that cannot allocate,
// such as code under HIP graph capture.
//
// It computes what tlim_spectral_bound computes -- lambda_G = max_i 2 d_i /
// C_i with d_i = sum_f w_f Lambda_f (Sec. 3.2 needs lambda_max of L_h; the
// faces of eq. qk_dis) at the state after the temperature relaxation of
// Sec. 3.4.1 -- with the same device functions and the same operation order,
// from the caller's fields.  The relaxation acts cell by cell, so each cell
// relaxes itself and its neighbours on the fly instead of writing a relaxed
// copy of the fields.  The only scratch is the row of reduction slots below,
// a file-scope device array held by every GPU the library runs on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tlim_device.h"
#include "tlim_internal.h"

namespace tlim {

namespace {

constexpr int kNaSlots = 256;  // reduction slots: the whole scratch (2 KiB per device)
constexpr int kNaDevices = 64;

// Scratch of the allocation-free bound.  In host code this name is only a
// handle for hipGetSymbolAddress; kernels get the device address.
static __device__ __align__(256) double scratch[kNaSlots];

__global__ void __launch_bounds__(kNaSlots) k_na_clear(double* slots) { slots[threadIdx.x] = 0.0; }

struct NaIn {
    const double *alpha2, *m1, *m2, *T1, *T2;
};

// Lambda and 1/C of cell a at its relaxed state.
__device__ __forceinline__ void relaxed_coef(const DevPhases& ph, double eps, const NaIn& in, int64_t a, double& L,
                                             double& r) {
    double T, a2;
    const double m1 = in.m1[a], m2 = in.m2[a];
    phys::relax_cell(ph, eps, in.alpha2[a], in.T1[a], in.T2[a], m1, m2, T, a2);
    L = phys::cell_conductivity(ph, T, a2, m1 + m2);
    r = phys::inv_heat_capacity(ph, eps, T, a2, m1, m2);
}

// 2 d_i / C_i of every cell, max into slot (wave % kNaSlots); faces in the
// order -x, +x, -y, +y, -z, +z.
__global__ void __launch_bounds__(256) k_na_bound(DevGrid g, DevPhases ph, double eps, int face, NaIn in,
                                                  double* slots) {
    double bound = 0.0;
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t st[3] = {1, g.nx, plane};
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < g.N; a += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(a / plane);
        const int64_t rest = a - (int64_t)k * plane;
        const int j = (int)(rest / g.nx);
        const int i = (int)(rest - (int64_t)j * g.nx);
        const int c[3] = {i, j, k};
        double L, r;
        relaxed_coef(ph, eps, in, a, L, r);
        double d = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (n[ax] <= 1) continue;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool inner = side ? c[ax] < n[ax] - 1 : c[ax] > 0;
                if (!inner && !g.per[ax]) continue;  // an adiabatic end has no face
                const int64_t off = inner ? (side ? st[ax] : -st[ax])
                                          : (side ? -(int64_t)(n[ax] - 1) * st[ax] : (int64_t)(n[ax] - 1) * st[ax]);
                double Lb, rb;
                relaxed_coef(ph, eps, in, a + off, Lb, rb);
                d += g.w[ax] * tb::fmean<double>(L, Lb, face);
            }
        }
        bound = fmax(bound, 2.0 * d * r);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bound = fmax(bound, __shfl_xor(bound, o, 64));
    if ((threadIdx.x & 63) == 0) {
        const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        atomicMax((unsigned long long*)(slots + w % kNaSlots),
                  (unsigned long long)__double_as_longlong(bound + 0.0));
    }
}

__global__ void __launch_bounds__(64) k_na_fold(const double* slots, double* out) {
    double m = 0.0;
    for (int s = threadIdx.x; s < kNaSlots; s += 64) m = fmax(m, slots[s]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (threadIdx.x == 0) out[0] = m;
}

// Device address of `scratch` on each device, looked up once per device with
// that device current.
std::mutex na_mutex;
double* na_ptr[kNaDevices];

hipError_t scratch_of(int dev, double** out) {
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        na_ptr[dev] = (double*)p;
    }
    *out = na_ptr[dev];
    return hipSuccess;
}

tlim_status bad(tlim_status st, const char* msg) {
    set_free_error(msg);
    return st;
}

}  // namespace
}  // namespace tlim

extern "C" tlim_status tlim_spectral_bound_noalloc(const tlim_grid* grid, const tlim_phase phases[2],
                                                   int32_t face_mean, double alpha_eps, const double* alpha2_dev,
                                                   const double* m1_dev, const double* m2_dev, const double* T1_dev,
                                                   const double* T2_dev, double* lambda_dev, void* hip_stream) {
    using namespace tlim;
    if (const char* why = check_grid(grid)) return bad(TLIM_E_ARG, why);
    const int64_t N = grid->n[0] * grid->n[1] * grid->n[2];
    if (N > ((int64_t)1 << 31) - 1) return bad(TLIM_E_ARG, "grid larger than the allocation-free bound's limit of 2^31 - 1 cells");
    if (!phases) return bad(TLIM_E_ARG, "phases is NULL");
    for (int k = 0; k < 2; ++k)
        if (const char* why = check_phase(&phases[k])) return bad(TLIM_E_ARG, why);
    if (face_mean < 0 || face_mean > 1) return bad(TLIM_E_ARG, "unknown face_mean");
    if (!(alpha_eps >= 0.0 && alpha_eps < 0.5)) return bad(TLIM_E_ARG, "alpha_eps out of [0, 0.5)");
    if (!alpha2_dev || !m1_dev || !m2_dev || !T1_dev || !T2_dev || !lambda_dev)
        return bad(TLIM_E_ARG, "a field or the output pointer is NULL");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bad(TLIM_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kNaDevices) return bad(TLIM_E_ARG, "device index beyond the library's table of 64");
    double* slots = nullptr;
    const hipError_t e = scratch_of(dev, &slots);
    if (e != hipSuccess) return bad(TLIM_E_HIP, hipGetErrorString(e));
    const hipStream_t s = (hipStream_t)hip_stream;
    const DevGrid g = pack_grid(grid);
    const DevPhases ph = pack_phases(phases);
    const NaIn in{alpha2_dev, m1_dev, m2_dev, T1_dev, T2_dev};
    const int64_t want = (N + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(kNaSlots), 0, s, slots);
    hipLaunchKernelGGL(k_na_bound, dim3(blocks), dim3(256), 0, s, g, ph, alpha_eps, face_mean, in, slots);
    hipLaunchKernelGGL(k_na_fold, dim3(1), dim3(64), 0, s, slots, lambda_dev);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return bad(TLIM_E_HIP, hipGetErrorString(le));
    set_free_error("");
    return TLIM_OK;
}
