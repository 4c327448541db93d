// Lorenz-96 ensemble forecast for the cycling filter (Section 4), gfx950.
// One workgroup per member: the member's state lives in registers (PER
// elements per thread, the smallest power of two that holds it), each
// Runge-Kutta stage is published to LDS so every thread can read its cyclic
// neighbours, then the stage tendency is formed in registers. One barrier per
// stage, four stages per step.
#include <atomic>
#include <cmath>

#include "enkf_internal.h"
#include "enkf_l96.h"

namespace enkf {
namespace {

constexpr int L96_NT = 256;
constexpr int L96_PER_MAX = ENKF_L96_MAX_STATE / L96_NT;

// PER state elements per thread (n <= 256 PER). The stage inputs alternate
// between two LDS arrays, so one barrier per stage separates the writes of a
// stage from the reads of the previous one.
template <int PER>
__global__ __launch_bounds__(L96_NT) void l96_rk4_kernel(int n, double* __restrict__ X, int64_t ldx, int nsteps,
                                                         double F, double dt) {
  extern __shared__ double ys[];                  // [2][n]
  double* __restrict__ x = X + (int64_t)blockIdx.x * ldx;
  const int t = threadIdx.x;
  double xv[PER], acc[PER], yv[PER];
  int im1[PER], im2[PER], ip1[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + q * L96_NT;
    xv[q] = i < n ? x[i] : 0.0;
    im1[q] = (i + n - 1) % n;
    im2[q] = (i + n - 2) % n;
    ip1[q] = (i + 1) % n;
  }
  const double h = 0.5 * dt;
  int buf = 0;
  for (int s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      yv[q] = xv[q];
      acc[q] = 0.0;
    }
#pragma unroll
    for (int stage = 0; stage < 4; ++stage) {
      double* __restrict__ y = ys + buf * n;
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (t + q * L96_NT < n) y[t + q * L96_NT] = yv[q];
      __syncthreads();
      const double w = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      const double c = stage == 2 ? dt : h;   // next stage input: x + c k
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = t + q * L96_NT;
        if (i < n) {
          const double k = (y[ip1[q]] - y[im2[q]]) * y[im1[q]] - y[i] + F;
          acc[q] += w * k;
          yv[q] = xv[q] + c * k;
        }
      }
      buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) xv[q] += dt / 6.0 * acc[q];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if (t + q * L96_NT < n) x[t + q * L96_NT] = xv[q];
}

template <int PER>
enkf_status l96_go(int n, int m, double* X, int64_t ldx, int nsteps, double F, double dt, hipStream_t s) {
  const size_t lds = 2 * sizeof(double) * (size_t)n;
  static std::atomic<uint64_t> attr{0};
  enkf_status st = set_dynamic_lds(attr, (const void*)l96_rk4_kernel<PER>, 2 * sizeof(double) * L96_NT * PER,
                                   "l96_forecast: cannot set the LDS size");
  if (st != ENKF_SUCCESS) return st;
  l96_rk4_kernel<PER><<<(unsigned)m, L96_NT, lds, s>>>(n, X, ldx, nsteps, F, dt);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
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
  const int n = (int)n_state;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int per = (n + L96_NT - 1) / L96_NT;
  if (per <= 1) return l96_go<1>(n, m, X, ldx, nsteps, F, dt, s);
  if (per <= 2) return l96_go<2>(n, m, X, ldx, nsteps, F, dt, s);
  if (per <= 4) return l96_go<4>(n, m, X, ldx, nsteps, F, dt, s);
  if (per <= 8) return l96_go<8>(n, m, X, ldx, nsteps, F, dt, s);
  if (per <= 16) return l96_go<16>(n, m, X, ldx, nsteps, F, dt, s);
  return l96_go<L96_PER_MAX>(n, m, X, ldx, nsteps, F, dt, s);
}
