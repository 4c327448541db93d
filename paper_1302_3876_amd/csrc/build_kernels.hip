// Build of the solve's inputs from the ensemble (Section 3, eq.
// system-rewritten), for gfx950: each observation's row of X^B is gathered,
// its member mean formed in FP64, and the scaled anomalies V and the
// innovations D written.
#include <algorithm>
#include <cmath>

#include "enkf_internal.h"

namespace enkf {
namespace {

// ------------------------------------------------------------------- build
// Block = 64 observations (lane) x 4 waves; wave w takes the members w,
// w + 4, ... of its lane's row. The member mean is the sum of the four wave
// partials, added in a fixed order.
constexpr int BV_OBS = 64;
constexpr int BV_REG = 32;    // at most this many members per wave held in registers (N <= 128)

template <typename T>
__device__ __forceinline__ double bv_mean(double sum, int N) {
  __shared__ double part[4][BV_OBS];
  const int lane = threadIdx.x % BV_OBS, w = threadIdx.x / BV_OBS;
  part[w][lane] = sum;
  __syncthreads();
  return ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) / (double)N;
}

// N <= 128: one pass, the row's members stay in registers between the mean
// and the writes.
template <typename T, int Q>
__global__ __launch_bounds__(256) void build_vd_reg_kernel(int N, const T* __restrict__ XB, int64_t ldx,
                                                           const int64_t* __restrict__ obs, int64_t n_obs,
                                                           const double* __restrict__ y, const T* __restrict__ E,
                                                           int64_t lde, T* __restrict__ V, T* __restrict__ D,
                                                           int64_t ldv, double inv_sqrt) {
  const int lane = threadIdx.x % BV_OBS, w = threadIdx.x / BV_OBS;
  const int64_t i = (int64_t)blockIdx.x * BV_OBS + lane;
  const int64_t ic = min(i, n_obs - 1);
  const int64_t s = obs[ic];
  T x[Q], e[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {                  // members past N read the last one, unused
    const int j = min(w + 4 * q, N - 1);
    x[q] = XB[s + (int64_t)j * ldx];
    e[q] = E[ic + (int64_t)j * lde];
  }
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) sum += (w + 4 * q < N) ? (double)x[q] : 0.0;
  const double mean = bv_mean<T>(sum, N);
  const double yi = y[ic];
  if (i < n_obs) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = w + 4 * q;
      if (j < N) {
        V[i + (int64_t)j * ldv] = (T)(((double)x[q] - mean) * inv_sqrt);
        D[i + (int64_t)j * ldv] = (T)((yi + (double)e[q]) - (double)x[q]);
      }
    }
  }
}

// Any N: every block forms its 64 rows' means over all members (8 loads in
// flight per lane), then writes the members [blockIdx.y mc, + mc).
template <typename T>
__global__ __launch_bounds__(256) void build_vd_chunk_kernel(int N, int mc, const T* __restrict__ XB, int64_t ldx,
                                                             const int64_t* __restrict__ obs, int64_t n_obs,
                                                             const double* __restrict__ y, const T* __restrict__ E,
                                                             int64_t lde, T* __restrict__ V, T* __restrict__ D,
                                                             int64_t ldv, double inv_sqrt) {
  constexpr int U = 8;
  const int lane = threadIdx.x % BV_OBS, w = threadIdx.x / BV_OBS;
  const int64_t i = (int64_t)blockIdx.x * BV_OBS + lane;
  const int64_t ic = min(i, n_obs - 1);
  const int64_t s = obs[ic];
  double sum = 0.0;
  int j = w;
  for (; j + 4 * (U - 1) < N; j += 4 * U) {
    T x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = XB[s + (int64_t)(j + 4 * u) * ldx];
#pragma unroll
    for (int u = 0; u < U; ++u) sum += (double)x[u];
  }
  for (; j < N; j += 4) sum += (double)XB[s + (int64_t)j * ldx];
  const double mean = bv_mean<T>(sum, N);
  const double yi = y[ic];
  const int j0 = blockIdx.y * mc, j1 = min(N, j0 + mc);
  for (int jb = j0 + w; jb < j1; jb += 4 * U) {
    T x[U], e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {                 // members past the chunk read its last one, unused
      const int jj = min(jb + 4 * u, j1 - 1);
      x[u] = XB[s + (int64_t)jj * ldx];
      e[u] = E[ic + (int64_t)jj * lde];
    }
    if (i < n_obs) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = jb + 4 * u;
        if (jj < j1) {
          V[i + (int64_t)jj * ldv] = (T)(((double)x[u] - mean) * inv_sqrt);
          D[i + (int64_t)jj * ldv] = (T)((yi + (double)e[u]) - (double)x[u]);
        }
      }
    }
  }
}

template <typename T, int Q>
void build_reg_go(int64_t blocks, int N, const void* XB, int64_t ldx, const int64_t* obs, int64_t n_obs,
                  const double* y, const void* E, int64_t lde, void* V, void* D, int64_t ldv, double inv_sqrt,
                  hipStream_t s) {
  build_vd_reg_kernel<T, Q><<<(unsigned)blocks, 256, 0, s>>>(N, (const T*)XB, ldx, obs, n_obs, y, (const T*)E, lde,
                                                              (T*)V, (T*)D, ldv, inv_sqrt);
}

}  // namespace

enkf_status launch_build_vd(enkf_dtype dt, int64_t n_state, int n_ens, const void* XB, int64_t ldx,
                            const int64_t* obs_idx, int64_t n_obs, const double* y, const void* E, int64_t lde,
                            void* V, void* D, int64_t ldv, hipStream_t s) {
  (void)n_state;
  if (n_obs <= 0) return ENKF_SUCCESS;
  const double inv_sqrt = 1.0 / std::sqrt((double)(n_ens - 1));
  const int64_t blocks = (n_obs + BV_OBS - 1) / BV_OBS;
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "build: too many observations for the grid");
  if (n_ens <= 4 * BV_REG) {
    const int q = (n_ens + 3) / 4;                // members per wave
    if (dt == ENKF_F64) {
      if (q <= 8) build_reg_go<double, 8>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else if (q <= 16) build_reg_go<double, 16>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else if (q <= 24) build_reg_go<double, 24>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else build_reg_go<double, 32>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
    } else {
      if (q <= 8) build_reg_go<float, 8>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else if (q <= 16) build_reg_go<float, 16>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else if (q <= 24) build_reg_go<float, 24>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
      else build_reg_go<float, 32>(blocks, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, inv_sqrt, s);
    }
  } else {
    // enough member chunks for about 2048 blocks, each chunk >= 32 members
    const int64_t want = std::max<int64_t>(1, (2048 + blocks - 1) / blocks);
    const int chunks = (int)std::min<int64_t>(want, std::max(1, n_ens / 32));
    const int mc = (n_ens + chunks - 1) / chunks;
    dim3 grid((unsigned)blocks, (unsigned)((n_ens + mc - 1) / mc));
    if (dt == ENKF_F64)
      build_vd_chunk_kernel<double><<<grid, 256, 0, s>>>(n_ens, mc, (const double*)XB, ldx, obs_idx, n_obs, y,
                                                         (const double*)E, lde, (double*)V, (double*)D, ldv, inv_sqrt);
    else
      build_vd_chunk_kernel<float><<<grid, 256, 0, s>>>(n_ens, mc, (const float*)XB, ldx, obs_idx, n_obs, y,
                                                        (const float*)E, lde, (float*)V, (float*)D, ldv, inv_sqrt);
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
