// Inner LIM stages (eq. LIM): dispatch between the one-stage kernels and the
// temporally blocked ones.
#include <hip/hip_runtime.h>

#include "tlim_sweep.h"

namespace tlim {

int launch_sweeps64(hipStream_t s, const DevGrid& g, int face, const double* v, const double* rhs,
                    const double* Lam, const double* rC, double* out, const double* b, int count, double tau) {
    (void)count;
    double tb = tau * b[0];
    launch_stage64(s, g, face, v, rhs, Lam, rC, out, 1.0 / (1.0 + tb), tb, tau);
    return 1;
}

int launch_sweeps32(hipStream_t s, const DevGrid& g, int face, const float* w, const float* q,
                    const float* Lam32, const float* rC32, float* out, const double* b, int count, double tau) {
    (void)count;
    double tb = tau * b[0];
    launch_stage32(s, g, face, w, q, Lam32, rC32, out, (float)(1.0 / (1.0 + tb)), (float)tb, (float)tau);
    return 1;
}

}  // namespace tlim
