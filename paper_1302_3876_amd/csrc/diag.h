// Launchers of the solve diagnostics (diag_kernels.hip).
#pragma once

#include "enkf_internal.h"

namespace enkf {

// out[0] = max_i r_i + rq, rq the Rayleigh quotient of the N x N Gram
// G = V^T V after a fixed number of power steps (rq <= its largest
// eigenvalue, and close to it once the iteration has converged): an
// estimate of ||R + V V^T||_2 that is at most 2 ||W||_2 and, converged, at
// least ||W||_2. part holds wnorm_partial_elems() doubles; N <= wnorm_max_n_ens().
int wnorm_partial_elems();
int wnorm_max_n_ens();
enkf_status launch_wnorm_estimate(int64_t n, int N, const double* r, const double* G, int64_t ldg, double* part,
                                  double* out, hipStream_t s);

}  // namespace enkf
