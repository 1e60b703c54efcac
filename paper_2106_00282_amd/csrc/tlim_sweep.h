// Launchers of the inner LIM stages (eq. LIM, m = 1 .. 2P-2).  One call
// advances up to `count` consecutive stages with parameters b[0..count-1]
// and returns how many it did (>= 1); the result is in `out`.  Several
// stages per launch are fused where the grid and arithmetic allow
// (temporal blocking), otherwise one stage is launched.
#pragma once

#include "tlim_internal.h"

namespace tlim {

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, const double* b, int count, double tau);

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* q,
                    const float* Lam32, const float* rC32, float* out, const double* b, int count, double tau);

}  // namespace tlim
