// Build of the solve's inputs from the ensemble (Section 3, eq.
// system-rewritten), for gfx950: one thread per observation gathers its row
// of X^B, forms the member mean in FP64 and writes the scaled anomalies V and
// the innovations D.
#include "enkf_internal.h"

namespace enkf {
namespace {

// ------------------------------------------------------------------- build
template <typename T>
__global__ __launch_bounds__(256) void build_vd_kernel(int64_t n_state, int N, const T* __restrict__ XB, int64_t ldx,
                                                       const int64_t* __restrict__ obs, int64_t n_obs,
                                                       const double* __restrict__ y, const T* __restrict__ E,
                                                       int64_t lde, T* __restrict__ V, T* __restrict__ D,
                                                       int64_t ldv, double inv_sqrt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_obs) return;
  const int64_t s = obs[i];
  double sum = 0.0;
  for (int j = 0; j < N; ++j) sum += (double)XB[s + (int64_t)j * ldx];
  const double mean = sum / (double)N;
  const double yi = y[i];
  for (int j = 0; j < N; ++j) {
    const double x = (double)XB[s + (int64_t)j * ldx];
    V[i + (int64_t)j * ldv] = (T)((x - mean) * inv_sqrt);
    D[i + (int64_t)j * ldv] = (T)((yi + (double)E[i + (int64_t)j * lde]) - x);
  }
}

}  // namespace

enkf_status launch_build_vd(enkf_dtype dt, int64_t n_state, int n_ens, const void* XB, int64_t ldx,
                            const int64_t* obs_idx, int64_t n_obs, const double* y, const void* E, int64_t lde,
                            void* V, void* D, int64_t ldv, hipStream_t s) {
  const double inv_sqrt = 1.0 / std::sqrt((double)(n_ens - 1));
  const int64_t blocks = (n_obs + 255) / 256;
  if (dt == ENKF_F64)
    build_vd_kernel<double><<<(unsigned)blocks, 256, 0, s>>>(n_state, n_ens, (const double*)XB, ldx, obs_idx, n_obs, y,
                                                             (const double*)E, lde, (double*)V, (double*)D, ldv, inv_sqrt);
  else
    build_vd_kernel<float><<<(unsigned)blocks, 256, 0, s>>>(n_state, n_ens, (const float*)XB, ldx, obs_idx, n_obs, y,
                                                            (const float*)E, lde, (float*)V, (float*)D, ldv, inv_sqrt);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
