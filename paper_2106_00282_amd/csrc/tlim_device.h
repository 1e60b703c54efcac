// Device helpers shared by the temporally blocked 2D kernels (forward
// stages in tlim_sweep.hip, reverse stages in tlim_adjoint.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace tlim {
namespace tb {

// Extended tile: 64 lanes (x) by WAVES waves of ROWS rows (y) per workgroup;
// up to KMAX stages per launch.
constexpr int KMAX = 8;
constexpr int WAVES = 8;
constexpr int ROWS = 8;
constexpr int EXT_Y = WAVES * ROWS;

// Lane i receives lane i-1 (wave_shr:1) or lane i+1 (wave_shl:1); with
// bound_ctrl the lanes at the ends receive 0 (they are halo lanes).
static __device__ __forceinline__ int dpp_from_left(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true); }
static __device__ __forceinline__ int dpp_from_right(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true); }

static __device__ __forceinline__ double from_left(double x) {
    return __hiloint2double(dpp_from_left(__double2hiint(x)), dpp_from_left(__double2loint(x)));
}
static __device__ __forceinline__ double from_right(double x) {
    return __hiloint2double(dpp_from_right(__double2hiint(x)), dpp_from_right(__double2loint(x)));
}
static __device__ __forceinline__ float from_left(float x) { return __int_as_float(dpp_from_left(__float_as_int(x))); }
static __device__ __forceinline__ float from_right(float x) { return __int_as_float(dpp_from_right(__float_as_int(x))); }

template <typename R>
static __device__ __forceinline__ R fmean(R a, R b, int face) {
    if (face == 1) {
        R s = a + b;
        return s > R(0) ? R(2) * (a * b) / s : R(0);
    }
    return R(0.5) * (a + b);
}

// Index of an unwrapped coordinate: wrap on a periodic axis, clamp on an
// adiabatic one (clamped copies only feed halo cells, whose wall faces
// carry kappa = 0).
static __device__ __forceinline__ int fold(int c, int n, int per) {
    if (per) {
        int m = c % n;
        return m < 0 ? m + n : m;
    }
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

}  // namespace tb
}  // namespace tlim
