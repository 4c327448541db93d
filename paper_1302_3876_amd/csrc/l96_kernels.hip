// Lorenz-96 ensemble forecast for the cycling filter (Section 4), gfx950.
// One workgroup per member: the member's state lives in registers (up to
// L96_PER elements per thread), each Runge-Kutta stage is published to LDS so
// every thread can read its cyclic neighbours, then the stage tendency is
// formed in registers. Two barriers per stage, four stages per step.
#include <cmath>

#include "enkf_internal.h"
#include "enkf_l96.h"

namespace enkf {
namespace {

constexpr int L96_NT = 256;
constexpr int L96_PER = ENKF_L96_MAX_STATE / L96_NT;

__global__ __launch_bounds__(L96_NT) void l96_rk4_kernel(int n, double* __restrict__ X, int64_t ldx, int nsteps,
                                                         double F, double dt) {
  extern __shared__ double ys[];
  double* __restrict__ x = X + (int64_t)blockIdx.x * ldx;
  const int t = threadIdx.x;
  double xv[L96_PER], acc[L96_PER], yv[L96_PER];
  int im1[L96_PER], im2[L96_PER], ip1[L96_PER];
#pragma unroll
  for (int q = 0; q < L96_PER; ++q) {
    const int i = t + q * L96_NT;
    xv[q] = i < n ? x[i] : 0.0;
    im1[q] = (i + n - 1) % n;
    im2[q] = (i + n - 2) % n;
    ip1[q] = (i + 1) % n;
  }
  const double h = 0.5 * dt;
  for (int s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int q = 0; q < L96_PER; ++q) {
      yv[q] = xv[q];
      acc[q] = 0.0;
    }
#pragma unroll
    for (int stage = 0; stage < 4; ++stage) {
#pragma unroll
      for (int q = 0; q < L96_PER; ++q)
        if (t + q * L96_NT < n) ys[t + q * L96_NT] = yv[q];
      __syncthreads();
      const double w = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      const double c = stage == 2 ? dt : h;   // next stage input: x + c k
#pragma unroll
      for (int q = 0; q < L96_PER; ++q) {
        const int i = t + q * L96_NT;
        if (i < n) {
          const double k = (ys[ip1[q]] - ys[im2[q]]) * ys[im1[q]] - ys[i] + F;
          acc[q] += w * k;
          yv[q] = xv[q] + c * k;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < L96_PER; ++q) xv[q] += dt / 6.0 * acc[q];
  }
#pragma unroll
  for (int q = 0; q < L96_PER; ++q)
    if (t + q * L96_NT < n) x[t + q * L96_NT] = xv[q];
}

}  // namespace
}  // namespace enkf

using namespace enkf;

extern "C" enkf_status enkf_l96_forecast(int64_t n_state, int32_t m, double* X, int64_t ldx, int32_t nsteps, double F,
                                         double dt, void* stream) {
  if (n_state < 4 || m < 0 || nsteps < 0 || (m > 0 && (!X || ldx < n_state)) || !std::isfinite(F) ||
      !std::isfinite(dt))
    return fail(ENKF_ERR_INVALID_ARG, "l96_forecast: bad argument");
  if (n_state > ENKF_L96_MAX_STATE) return fail(ENKF_ERR_NOT_SUPPORTED, "l96_forecast: n_state above ENKF_L96_MAX_STATE");
  if (m == 0 || nsteps == 0) return ENKF_SUCCESS;
  const size_t lds = sizeof(double) * (size_t)n_state;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)l96_rk4_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(double) * ENKF_L96_MAX_STATE));
    attr = true;
  }
  l96_rk4_kernel<<<(unsigned)m, L96_NT, lds, static_cast<hipStream_t>(stream)>>>((int)n_state, X, ldx, nsteps, F, dt);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}
