// Pivoting of the plain sweeps (Section 3.4, eq. gamma-value), for gfx950.
//
// Before level k the paper picks, among the columns not used yet, the one
// whose pivot 1 + v_i^T u_i^{(k-1)} is largest in magnitude and swaps it into
// position k. Here nothing is moved: perm[k] is the V/U column used at level
// k, the level kernels follow perm and a list of the active columns, and the
// candidate pivots are kept up to date in O(N) per level instead of being
// recomputed with n-long products: after level k (pivot column p, pivot g)
//     g_i <- g_i - c_i^2 / g,     c_i = v_p^T u_i^{(k-1)} = v_i^T u_p^{(k-1)},
// since u_i^{(k)} = u_i^{(k-1)} - u_p c_i / g and W_{k-1}^{-1} is symmetric.
// The c_i are the products the previous launch already left (its look-ahead
// with v_p), so the selection costs no extra pass over the data. Initial
// candidates g_i = 1 + v_i^T R^{-1} v_i come from one pass over V.
#include "enkf_internal.h"

namespace enkf {
namespace {

constexpr int PV_THREADS = 256;
constexpr int PV_WAVES = PV_THREADS / kWave;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// The level kernels' fixed-order sum of one column of partials.
__device__ __forceinline__ double column_sum(const double* __restrict__ p, int nb, int lane) {
  double s = 0.0;
  int b = lane;
  for (; b + 3 * kWave < nb; b += 4 * kWave) {
    const double x0 = p[b], x1 = p[b + kWave], x2 = p[b + 2 * kWave], x3 = p[b + 3 * kWave];
    s += x0;
    s += x1;
    s += x2;
    s += x3;
  }
  for (; b < nb; b += kWave) s += p[b];
  return wave_sum(s);
}

// part[i * nb + b] = sum over the rows of block b of V[row, i]^2 / r[row].
template <typename T>
__global__ __launch_bounds__(PV_THREADS) void diag_partial_kernel(int64_t n, const T* __restrict__ V, int64_t ldv,
                                                                  const double* __restrict__ r, int64_t rows_per_block,
                                                                  double* __restrict__ part) {
  __shared__ double red[PV_WAVES];
  const int i = blockIdx.y, nb = gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  const T* __restrict__ v = V + (int64_t)i * ldv;
  double s = 0.0;
  for (int64_t row = r0 + threadIdx.x; row < r1; row += PV_THREADS) {
    const double x = (double)v[row];
    s += x * x / r[row];
  }
  s = wave_sum(s);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PV_WAVES; ++w) t += red[w];
    part[(int64_t)i * nb + blockIdx.x] = t;
  }
}

// Index (into cand) of the largest key over the block, ties to the smaller
// index; every thread passes its best (key, index) pair.
__device__ __forceinline__ int block_argmax(double key, int idx, double* kbuf, int* ibuf) {
  const int t = threadIdx.x;
  kbuf[t] = key;
  ibuf[t] = idx;
  __syncthreads();
  for (int s = PV_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double k2 = kbuf[t + s];
      const int i2 = ibuf[t + s];
      if (i2 >= 0 && (ibuf[t] < 0 || k2 > kbuf[t] || (k2 == kbuf[t] && i2 < ibuf[t]))) {
        kbuf[t] = k2;
        ibuf[t] = i2;
      }
    }
    __syncthreads();
  }
  const int best = ibuf[0];
  __syncthreads();
  return best;
}

// One block. init: candidates from the diagonal partials, perm[0], rem_out =
// 0..N-1. Level k: c_i for the remaining columns from the look-ahead partials,
// gamma[k] = 1 + c_p (p = perm[k]); the active list of level k (remaining
// columns without p, in order, then the nz Z columns N..N+nz-1); candidate
// update; perm[k+1].
__global__ __launch_bounds__(PV_THREADS) void pivot_kernel(PivotArgs a) {
  __shared__ double kbuf[PV_THREADS];
  __shared__ int ibuf[PV_THREADS];
  __shared__ int pos_s;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int N = a.N;
  if (a.init) {
    for (int i = wave; i < N; i += PV_WAVES) {
      const double d = column_sum(a.part + (int64_t)i * a.nb, a.nb, lane);
      if (lane == 0) a.gcur[i] = 1.0 + d;
    }
    __syncthreads();
    double bk = 0.0;
    int bi = -1;
    for (int i = t; i < N; i += PV_THREADS) {
      const double g = a.gcur[i];
      a.rem_out[i] = i;
      if (bi < 0 || g > bk) { bk = g; bi = i; }
    }
    const int best = block_argmax(bk, bi, kbuf, ibuf);
    if (t == 0) a.perm[0] = best;
    return;
  }
  const int k = a.k;
  const int nr = N - k;                 // remaining columns, including p
  const int p = a.perm[k];
  for (int j = wave; j < nr; j += PV_WAVES) {
    const int id = a.rem_in[j];
    const double c = column_sum(a.part + (int64_t)id * a.nb, a.nb, lane);
    if (lane == 0) a.cbuf[id] = c;
  }
  if (t == 0) pos_s = 0;
  __syncthreads();
  for (int j = t; j < nr; j += PV_THREADS)
    if (a.rem_in[j] == p) pos_s = j;
  __syncthreads();
  const int pos = pos_s;
  const double gp = 1.0 + a.cbuf[p];
  if (t == 0) {
    a.gamma[k] = gp;
    if (!(gp > 0.0) || !__builtin_isfinite(gp)) atomicOr(a.status, kStatusNotSpd);
  }
  const double inv = 1.0 / gp;
  double bk = 0.0;
  int bi = -1;
  for (int j = t; j < nr - 1; j += PV_THREADS) {
    const int id = a.rem_in[j < pos ? j : j + 1];
    a.act_out[j] = id;
    a.rem_out[j] = id;
    const double c = a.cbuf[id];
    const double g = a.gcur[id] - c * c * inv;
    a.gcur[id] = g;
    if (bi < 0 || g > bk) { bk = g; bi = j; }
  }
  for (int z = t; z < a.nz; z += PV_THREADS) a.act_out[nr - 1 + z] = N + z;
  if (k + 1 < N) {
    const int best = block_argmax(bk, bi, kbuf, ibuf);
    if (t == 0) a.perm[k + 1] = a.rem_in[best < pos ? best : best + 1];
  }
}

}  // namespace

enkf_status launch_diag_partials(enkf_dtype dt, int64_t n, int N, const void* V, int64_t ldv, const double* r,
                                 int nb, double* part, hipStream_t s) {
  if (N > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "pivoting: more than 65535 members");
  const int64_t rpb = (n + nb - 1) / nb;
  dim3 grid((unsigned)nb, (unsigned)N);
  if (dt == ENKF_F64)
    diag_partial_kernel<double><<<grid, PV_THREADS, 0, s>>>(n, static_cast<const double*>(V), ldv, r, rpb, part);
  else
    diag_partial_kernel<float><<<grid, PV_THREADS, 0, s>>>(n, static_cast<const float*>(V), ldv, r, rpb, part);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_pivot(const PivotArgs& a, hipStream_t s) {
  pivot_kernel<<<1, PV_THREADS, 0, s>>>(a);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
