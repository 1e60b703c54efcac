// Launchers of the LIM stages (eq. LIM).  One call advances up to `count`
// consecutive stages with parameters b[0..count-1] and returns how many it
// did (>= 1, = sweeps_per_launch(g, count)); the result is in `out`.  Several
// stages per launch are fused where the grid allows (temporal blocking),
// otherwise one stage is launched.  In FP64 the final stage (b = 0) may be
// among them; the FP32 correction form finishes with launch_final32.  The FP32
// source is qn = -tau A' g.
#pragma once

#include "tlim_internal.h"

namespace tlim {

// Number of stages the next launch will advance when `count` remain.
int sweeps_per_launch(const DevGrid& g, int count);

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, const double* b, int count, double tau);

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* qn,
                    const float* Lam32, const float* rC32, float* out, const double* b, int count, double tau);

}  // namespace tlim
