// Launchers of the LIM stages (eq. LIM).  One call advances up to `count`
// consecutive stages and returns how many it did (>= 1, equal to
// sweeps_per_launch(g, count)); the result is in `out`.  Several stages per
// launch are fused where the grid allows (temporal blocking), otherwise one
// stage is launched.  In FP64 the final stage (b = 0, flux form) may be among
// them: a launch with last = true ends the pass and, when Tit != NULL, also
// accumulates the pass reductions (dmax, tmax, bad) into ps.  The FP32
// correction form advances inner stages only (source qn = -tau A' g) and
// finishes with launch_final32.
#pragma once

#include "tlim_internal.h"

namespace tlim {

// Parameters of consecutive stages (host arrays, already offset to the first
// stage of the launch): with lam == NULL stage k uses tau*b_k = tb[k];
// otherwise tau*b_k = tau * (*lam) * chat[k], lam pointing to device memory.
struct Stages {
    const double* lam;
    const double* tb;
    const double* chat;
};

// Number of stages the next launch will advance when `count` remain.
int sweeps_per_launch(const DevGrid& g, int count);

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, Stages st, int count, bool last, double tau,
                    const double* Tit, PassSlots ps);

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* qn,
                    const float* Lam32, const float* rC32, float* out, Stages st, int count, double tau);

}  // namespace tlim
