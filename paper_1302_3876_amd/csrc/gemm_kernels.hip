// Products around the solve, for gfx950:
//   - build of V and D from the ensemble (Section 3, eq. system-rewritten);
//   - the split-K product G = A^T B over the n observations (G = V^T Z of the
//     analysis update), reduced over row chunks in a fixed order;
//   - the analysis update X^A = X^B + (X^B - xbar 1^T) Gs (Section 3.1),
//     Gs = (V^T Z)/sqrt(N-1), as an LDS-tiled tall product whose prologue
//     subtracts the ensemble mean.
// Accumulation is FP64 for both storage types.
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

// ------------------------------------------------------------ split-K A^T B
constexpr int GR_TILE = 32;   // output tile GR_TILE x GR_TILE
constexpr int GR_SUB = 64;    // rows staged in LDS per step
constexpr int GR_THREADS = 256;

int64_t gram_chunks(int64_t n, int a, int m) {
  const int64_t tiles = (int64_t)((a + GR_TILE - 1) / GR_TILE) * ((m + GR_TILE - 1) / GR_TILE);
  int64_t chunks = (2048 + tiles - 1) / tiles;
  const int64_t max_chunks = (n + GR_SUB - 1) / GR_SUB;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  return chunks;
}

template <typename T>
__global__ __launch_bounds__(GR_THREADS) void gram_partial_kernel(int64_t n, int a, int m, const T* __restrict__ A,
                                                                  int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                                  double* __restrict__ partial, int64_t rows_per_chunk) {
  __shared__ double As[GR_SUB][GR_TILE + 1];
  __shared__ double Bs[GR_SUB][GR_TILE + 1];
  const int tiles_m = (m + GR_TILE - 1) / GR_TILE;
  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * GR_TILE, m0 = tm * GR_TILE;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x;
  // thread owns outputs (ia, jm), (ia+16, jm), (ia, jm+16), (ia+16, jm+16)
  const int ia = t % 16, jm = t / 16;
  double acc00 = 0, acc01 = 0, acc10 = 0, acc11 = 0;
  for (int64_t rs = r0; rs < r1; rs += GR_SUB) {
    // stage GR_SUB rows of the A and B column tiles (coalesced along rows)
    for (int e = t; e < GR_SUB * GR_TILE; e += GR_THREADS) {
      const int rr = e % GR_SUB, cc = e / GR_SUB;
      const int64_t row = rs + rr;
      const bool rok = row < r1;
      As[rr][cc] = (rok && a0 + cc < a) ? (double)A[row + (int64_t)(a0 + cc) * lda] : 0.0;
      Bs[rr][cc] = (rok && m0 + cc < m) ? (double)B[row + (int64_t)(m0 + cc) * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < GR_SUB; ++rr) {
      const double x0 = As[rr][ia], x1 = As[rr][ia + 16];
      const double y0 = Bs[rr][jm], y1 = Bs[rr][jm + 16];
      acc00 += x0 * y0; acc01 += x0 * y1; acc10 += x1 * y0; acc11 += x1 * y1;
    }
    __syncthreads();
  }
  double* P = partial + (int64_t)blockIdx.x * a * m;
  if (a0 + ia < a && m0 + jm < m) P[(a0 + ia) + (int64_t)(m0 + jm) * a] = acc00;
  if (a0 + ia < a && m0 + jm + 16 < m) P[(a0 + ia) + (int64_t)(m0 + jm + 16) * a] = acc01;
  if (a0 + ia + 16 < a && m0 + jm < m) P[(a0 + ia + 16) + (int64_t)(m0 + jm) * a] = acc10;
  if (a0 + ia + 16 < a && m0 + jm + 16 < m) P[(a0 + ia + 16) + (int64_t)(m0 + jm + 16) * a] = acc11;
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(int a, int m, int64_t chunks, const double* __restrict__ partial,
                                                          double* __restrict__ G, int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t am = (int64_t)a * m;
  if (e >= am) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += partial[c * am + e];
  const int i = (int)(e % a), j = (int)(e / a);
  G[i + (int64_t)j * ldg] = s;
}

// --------------------------------------------------------------- analysis
constexpr int AN_TR = 64, AN_TC = 128, AN_TK = 16;

// Block computes X^A[rows, cols] for a 64 x 128 tile; thread owns 4 x 8.
// The block first forms the means of its 64 rows (the rows of S it needs).
template <typename T>
__global__ __launch_bounds__(256) void analysis_tile_kernel(int64_t n_state, int N, const T* __restrict__ XB,
                                                            int64_t ldx, const double* __restrict__ G, double scale,
                                                            T* __restrict__ XA, int64_t ldxa) {
  __shared__ double As[AN_TK][AN_TR + 1];
  __shared__ double Bs[AN_TK][AN_TC + 1];
  __shared__ double part[4][AN_TR];
  __shared__ double mean[AN_TR];
  const int64_t row0 = (int64_t)blockIdx.x * AN_TR;
  const int col0 = blockIdx.y * AN_TC;
  const int t = threadIdx.x;
  {  // row means: 4 threads per row, members split in a fixed pattern
    const int rr = t % AN_TR, q = t / AN_TR;
    const int64_t row = row0 + rr;
    double sum = 0.0;
    if (row < n_state)
      for (int j = q; j < N; j += 4) sum += (double)XB[row + (int64_t)j * ldx];
    part[q][rr] = sum;
    __syncthreads();
    if (t < AN_TR) mean[t] = (((part[0][t] + part[1][t]) + part[2][t]) + part[3][t]) / (double)N;
    __syncthreads();
  }
  const int tr = t % 16, tc = t / 16;
  double acc[4][8] = {};
  for (int k0 = 0; k0 < N; k0 += AN_TK) {
    for (int e = t; e < AN_TK * AN_TR; e += 256) {
      const int rr = e % AN_TR, kk = e / AN_TR;
      const int64_t row = row0 + rr;
      As[kk][rr] = (row < n_state && k0 + kk < N) ? (double)XB[row + (int64_t)(k0 + kk) * ldx] - mean[rr] : 0.0;
    }
    for (int e = t; e < AN_TK * AN_TC; e += 256) {
      const int kk = e % AN_TK, cc = e / AN_TK;
      Bs[kk][cc] = (k0 + kk < N && col0 + cc < N) ? G[(k0 + kk) + (int64_t)(col0 + cc) * N] * scale : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < AN_TK; ++kk) {
      double a4[4], b8[8];
#pragma unroll
      for (int p = 0; p < 4; ++p) a4[p] = As[kk][tr + 16 * p];
#pragma unroll
      for (int q = 0; q < 8; ++q) b8[q] = Bs[kk][tc + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[p][q] += a4[p] * b8[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t row = row0 + tr + 16 * p;
    if (row >= n_state) continue;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = col0 + tc + 16 * q;
      if (col < N) XA[row + (int64_t)col * ldxa] = (T)((double)XB[row + (int64_t)col * ldx] + acc[p][q]);
    }
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

int64_t gram_partial_elems(int64_t n, int a, int m) { return gram_chunks(n, a, m) * (int64_t)a * m; }

enkf_status launch_gram(enkf_dtype dt, int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb,
                        double* G, int64_t ldg, double* partial, hipStream_t s) {
  if (a <= 0 || m <= 0) return ENKF_SUCCESS;
  const int64_t chunks = gram_chunks(n, a, m);
  int64_t rpc = (n + chunks - 1) / chunks;
  rpc = ((rpc + GR_SUB - 1) / GR_SUB) * GR_SUB;
  const int64_t used = (n + rpc - 1) / rpc;
  const int tiles = ((a + GR_TILE - 1) / GR_TILE) * ((m + GR_TILE - 1) / GR_TILE);
  dim3 grid((unsigned)used, (unsigned)tiles);
  if (dt == ENKF_F64)
    gram_partial_kernel<double><<<grid, GR_THREADS, 0, s>>>(n, a, m, (const double*)A, lda, (const double*)B, ldb,
                                                            partial, rpc);
  else
    gram_partial_kernel<float><<<grid, GR_THREADS, 0, s>>>(n, a, m, (const float*)A, lda, (const float*)B, ldb,
                                                           partial, rpc);
  ENKF_HIP_CHECK(hipGetLastError());
  const int64_t am = (int64_t)a * m;
  gram_reduce_kernel<<<(unsigned)((am + 255) / 256), 256, 0, s>>>(a, m, used, partial, G, ldg);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_analysis(enkf_dtype dt, int64_t n_state, int N, const void* XB, int64_t ldx, const double* G,
                            double scale, void* XA, int64_t ldxa, hipStream_t s) {
  dim3 grid((unsigned)((n_state + AN_TR - 1) / AN_TR), (unsigned)((N + AN_TC - 1) / AN_TC));
  if (dt == ENKF_F64)
    analysis_tile_kernel<double><<<grid, 256, 0, s>>>(n_state, N, (const double*)XB, ldx, G, scale, (double*)XA, ldxa);
  else
    analysis_tile_kernel<float><<<grid, 256, 0, s>>>(n_state, N, (const float*)XB, ldx, G, scale, (float*)XA, ldxa);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
