// Diagnostics of a solve (gfx950): the estimate of ||W||_2 = ||R + V V^T||_2
// that the normwise backward error divides by,
//   ||W||_2 <= max r + sigma_max(V)^2 <= 2 ||W||_2
// (both terms are positive semidefinite, Weyl's inequality), with
// sigma_max(V)^2 the largest eigenvalue of the N x N Gram V^T V taken by
// power iteration (the Rayleigh quotient of the last iterate, which never
// exceeds it).
#include "diag.h"

namespace enkf {
namespace {

constexpr int RMAX_BLOCKS = 256;
constexpr int PW_THREADS = 1024;
constexpr int PW_ITERS = 60;

__global__ __launch_bounds__(256) void rmax_partial_kernel(int64_t n, const double* __restrict__ r,
                                                           double* __restrict__ part) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmax(m, r[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Sum over the block of 1024 threads (16 waves) in a fixed order.
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < PW_THREADS / 64; ++w) s += red[w];
  return s;
}

// One block: x in the LDS, y = G x row by row (thread t: rows t + 1024 q;
// for a fixed column the threads read consecutive rows), then x = y / ||y||.
__global__ __launch_bounds__(PW_THREADS) void wnorm_kernel(int N, const double* __restrict__ G, int64_t ldg, int nb,
                                                           const double* __restrict__ part, double* __restrict__ out) {
  extern __shared__ double sh[];
  double* x = sh;
  double* y = sh + N;
  __shared__ double red[PW_THREADS / 64];
  const int t = threadIdx.x;
  // start: a positive, non-constant vector (the anomalies' Gram annihilates
  // the constant vector when the columns of V sum to zero)
  for (int j = t; j < N; j += PW_THREADS) {
    const double f = (double)j * 0.6180339887498949;
    x[j] = 0.5 + (f - floor(f));
  }
  __syncthreads();
  double rq = 0.0;
  for (int it = 0; it < PW_ITERS; ++it) {
    double xy = 0.0, yy = 0.0, xx = 0.0;
    for (int i = t; i < N; i += PW_THREADS) {
      double s = 0.0;
      for (int j = 0; j < N; ++j) s = fma(G[i + (int64_t)j * ldg], x[j], s);
      y[i] = s;
      xy = fma(x[i], s, xy);
      yy = fma(s, s, yy);
      xx = fma(x[i], x[i], xx);
    }
    xy = block_sum(xy, red);
    yy = block_sum(yy, red);
    xx = block_sum(xx, red);
    rq = xx > 0.0 ? xy / xx : 0.0;
    const double inv = yy > 0.0 ? 1.0 / sqrt(yy) : 0.0;
    __syncthreads();
    for (int i = t; i < N; i += PW_THREADS) x[i] = y[i] * inv;
    __syncthreads();
    if (yy == 0.0) break;
  }
  if (t == 0) {
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, part[b]);
    out[0] = m + rq;
  }
}

}  // namespace

int wnorm_partial_elems() { return RMAX_BLOCKS; }
int wnorm_max_n_ens() { return 4096; }

enkf_status launch_wnorm_estimate(int64_t n, int N, const double* r, const double* G, int64_t ldg, double* part,
                                  double* out, hipStream_t s) {
  if (N < 1 || N > wnorm_max_n_ens()) return fail(ENKF_ERR_NOT_SUPPORTED, "norm estimate: n_ens outside [1, 4096]");
  int nb = (int)((n + 255) / 256);
  if (nb > RMAX_BLOCKS) nb = RMAX_BLOCKS;
  if (nb < 1) nb = 1;
  rmax_partial_kernel<<<nb, 256, 0, s>>>(n, r, part);
  ENKF_HIP_CHECK(hipGetLastError());
  wnorm_kernel<<<1, PW_THREADS, 2 * sizeof(double) * (size_t)N, s>>>(N, G, ldg, nb, part, out);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
