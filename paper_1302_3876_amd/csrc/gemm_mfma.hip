// Matrix-core products of the blocked solve, the refinement residual and the
// analysis update, for gfx950.
//
//  tn: P = A^T B over the n observations, A: n x a, B: n x m, column-major,
//      split over row chunks; every chunk writes an a x m partial and a
//      second kernel sums the partials in chunk order (deterministic).
//      (the panel products V_K^T [U_K, X] of the Woodbury identity, eq. SWM,
//      and G = V^T Z of the analysis and of the residual)
//  nn: tall products with a short inner dimension K, column tiles of 64:
//      UPDATE    X   <- X - A Bm                 (X -= U_K Q, the panel update)
//      ANALYSIS  XA  <- XB + (XB - xbar 1^T)(s Bm) (X^A = X^B + S V^T Z, Section 3.1)
//      RESIDUAL  RHO <- D - (r o Z + A Bm)       (D - W Z with Bm = V^T Z)
//      Bm is FP64 (it comes from the FP64 panel factorisation or from the
//      FP64 products) and is rounded to the MFMA input type when staged.
// Tiles are staged through LDS with coalesced column reads; the MFMA result
// lanes run along rows, so stores are coalesced as well.
#include "enkf_internal.h"
#include "gemm_mfma.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int NT = 256;  // 4 waves

template <typename T> struct MfOf;
template <> struct MfOf<double> { typedef MfmaF64 type; };
template <> struct MfOf<float> { typedef MfmaF32 type; };

// ---------------------------------------------------------------- tn
constexpr int TN_TA = 64, TN_TM = 64, TN_KC = 32, TN_PAD = 1;

template <typename T>
__global__ __launch_bounds__(NT) void tn_partial_kernel(int64_t n, int a, int m, const T* __restrict__ A, int64_t lda,
                                                        const T* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ partial, int64_t rows_per_chunk) {
  typedef typename MfOf<T>::type MF;
  __shared__ T As[TN_KC][TN_TA + TN_PAD];
  __shared__ T Bs[TN_KC][TN_TM + TN_PAD];
  const int tiles_m = (m + TN_TM - 1) / TN_TM;
  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * TN_TA, m0 = tm * TN_TM;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int m_off = (w / 2) * 32, a_off = (w % 2) * 32;
  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();

  for (int64_t rs = r0; rs < r1; rs += TN_KC) {
#pragma unroll 4
    for (int e = t; e < TN_KC * TN_TA; e += NT) {
      const int rr = e % TN_KC, cc = e / TN_KC;
      const int64_t row = rs + rr;
      As[rr][cc] = (row < r1 && a0 + cc < a) ? A[row + (int64_t)(a0 + cc) * lda] : T(0);
    }
#pragma unroll 4
    for (int e = t; e < TN_KC * TN_TM; e += NT) {
      const int rr = e % TN_KC, cc = e / TN_KC;
      const int64_t row = rs + rr;
      Bs[rr][cc] = (row < r1 && m0 + cc < m) ? B[row + (int64_t)(m0 + cc) * ldb] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TN_KC; k += MF::KSTEP) {
      T bop[2], aop[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) bop[i] = Bs[k + l / 16][m_off + 16 * i + l % 16];
#pragma unroll
      for (int j = 0; j < 2; ++j) aop[j] = As[k + l / 16][a_off + 16 * j + l % 16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MF::mma(bop[i], aop[j], acc[i][j]);
    }
    __syncthreads();
  }
  // acc[i][j] element (row = m index, col = a index)
  double* P = partial + (int64_t)blockIdx.x * a * m;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mi = m0 + m_off + 16 * i + MF::row(l, r);
        const int ai = a0 + a_off + 16 * j + l % 16;
        if (mi < m && ai < a) P[ai + (int64_t)mi * a] = (double)acc[i][j][r];
      }
}

__global__ __launch_bounds__(256) void partial_sum_kernel(int a, int m, int64_t chunks, const double* __restrict__ partial,
                                                          double* __restrict__ G, int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t am = (int64_t)a * m;
  if (e >= am) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += partial[c * am + e];
  const int i = (int)(e % a), j = (int)(e / a);
  G[i + (int64_t)j * ldg] = s;
}

// ---------------------------------------------------------------- nn
constexpr int NN_TR = 64, NN_TC = 64, NN_KC = 16, NN_PAD = 1;

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void nn_kernel(NnArgs p) {
  typedef typename MfOf<T>::type MF;
  __shared__ T As[NN_KC][NN_TR + NN_PAD];   // As[k][row] = A[row, k] (- mean)
  __shared__ T Bs[NN_KC][NN_TC + NN_PAD];   // Bs[k][col] = s * Bm[k, col]
  __shared__ double mean[NN_TR];
  int64_t rt;
  int ct;
  xcd_tile_map(blockIdx.x, p.n_row_tiles, p.n_col_tiles, &rt, &ct);
  if (rt >= p.n_row_tiles) return;
  const int64_t row0 = rt * NN_TR;
  const int col0 = ct * NN_TC;
  const T* __restrict__ A = static_cast<const T*>(p.A);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int c_off = (w / 2) * 32, r_off = (w % 2) * 32;

  if constexpr (MODE == NN_ANALYSIS) {
    // row means of the block's rows (4 threads per row, fixed order)
    __shared__ double part[4][NN_TR];
    const int rr = t % NN_TR, q = t / NN_TR;
    const int64_t row = row0 + rr;
    double s = 0.0;
    if (row < p.n)
      for (int j = q; j < p.K; j += 4) s += (double)A[row + (int64_t)j * p.lda];
    part[q][rr] = s;
    __syncthreads();
    if (t < NN_TR) mean[t] = (((part[0][t] + part[1][t]) + part[2][t]) + part[3][t]) / (double)p.K;
    __syncthreads();
  }

  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();

  for (int k0 = 0; k0 < p.K; k0 += NN_KC) {
#pragma unroll 4
    for (int e = t; e < NN_KC * NN_TR; e += NT) {
      const int rr = e % NN_TR, kk = e / NN_TR;
      const int64_t row = row0 + rr;
      double v = 0.0;
      if (row < p.n && k0 + kk < p.K) {
        v = (double)A[row + (int64_t)(k0 + kk) * p.lda];
        if constexpr (MODE == NN_ANALYSIS) v -= mean[rr];
      }
      As[kk][rr] = (T)v;
    }
    for (int e = t; e < NN_KC * NN_TC; e += NT) {
      const int kk = e % NN_KC, cc = e / NN_KC;
      Bs[kk][cc] = (k0 + kk < p.K && col0 + cc < p.m) ? (T)(p.scale * p.Bm[(k0 + kk) + (int64_t)(col0 + cc) * p.ldb])
                                                       : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NN_KC; k += MF::KSTEP) {
      T cop[2], rop[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) cop[i] = Bs[k + l / 16][c_off + 16 * i + l % 16];
#pragma unroll
      for (int j = 0; j < 2; ++j) rop[j] = As[k + l / 16][r_off + 16 * j + l % 16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MF::mma(cop[i], rop[j], acc[i][j]);
    }
    __syncthreads();
  }
  // acc[i][j] element (row = output column, col = output row)
  const T* __restrict__ Cin = static_cast<const T*>(p.Cin);
  T* __restrict__ Cout = static_cast<T*>(p.Cout);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + c_off + 16 * i + MF::row(l, r);
        const int64_t row = row0 + r_off + 16 * j + l % 16;
        if (col < p.m && row < p.n) {
          const double prod = (double)acc[i][j][r];
          const double cin = (double)Cin[row + (int64_t)col * p.ldc];
          double out;
          if constexpr (MODE == NN_UPDATE) out = cin - prod;
          else if constexpr (MODE == NN_ANALYSIS) out = cin + prod;
          else out = (double)static_cast<const T*>(p.Din)[row + (int64_t)col * p.ldd] - (p.r[row] * cin + prod);
          Cout[row + (int64_t)col * p.ldo] = (T)out;
        }
      }
}

int64_t tn_chunks(int64_t n, int a, int m) {
  const int64_t tiles = (int64_t)((a + TN_TA - 1) / TN_TA) * ((m + TN_TM - 1) / TN_TM);
  int64_t chunks = (4096 + tiles - 1) / tiles;
  const int64_t max_chunks = (n + TN_KC - 1) / TN_KC;
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  return chunks;
}

}  // namespace

int64_t tn_partial_elems(int64_t n, int a, int m) { return tn_chunks(n, a, m) * (int64_t)a * m; }

enkf_status launch_tn(enkf_dtype dt, int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb,
                      double* G, int64_t ldg, double* partial, hipStream_t s) {
  if (a <= 0 || m <= 0) return ENKF_SUCCESS;
  const int64_t chunks = tn_chunks(n, a, m);
  int64_t rpc = (n + chunks - 1) / chunks;
  rpc = ((rpc + TN_KC - 1) / TN_KC) * TN_KC;
  const int64_t used = (n + rpc - 1) / rpc;
  const int tiles = ((a + TN_TA - 1) / TN_TA) * ((m + TN_TM - 1) / TN_TM);
  if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
  dim3 grid((unsigned)used, (unsigned)tiles);
  if (dt == ENKF_F64)
    tn_partial_kernel<double><<<grid, NT, 0, s>>>(n, a, m, (const double*)A, lda, (const double*)B, ldb, partial, rpc);
  else
    tn_partial_kernel<float><<<grid, NT, 0, s>>>(n, a, m, (const float*)A, lda, (const float*)B, ldb, partial, rpc);
  ENKF_HIP_CHECK(hipGetLastError());
  const int64_t am = (int64_t)a * m;
  partial_sum_kernel<<<(unsigned)((am + 255) / 256), 256, 0, s>>>(a, m, used, partial, G, ldg);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_nn(enkf_dtype dt, int mode, NnArgs p, hipStream_t s) {
  if (p.n <= 0 || p.m <= 0) return ENKF_SUCCESS;
  p.n_row_tiles = (p.n + NN_TR - 1) / NN_TR;
  p.n_col_tiles = (p.m + NN_TC - 1) / NN_TC;
  const int64_t groups = (p.n_row_tiles + 7) / 8;
  const int64_t blocks = groups * 8 * p.n_col_tiles;
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "nn product: grid too large");
  const unsigned g = (unsigned)blocks;
  if (dt == ENKF_F64) {
    if (mode == NN_UPDATE) nn_kernel<double, NN_UPDATE><<<g, NT, 0, s>>>(p);
    else if (mode == NN_ANALYSIS) nn_kernel<double, NN_ANALYSIS><<<g, NT, 0, s>>>(p);
    else nn_kernel<double, NN_RESIDUAL><<<g, NT, 0, s>>>(p);
  } else {
    if (mode == NN_UPDATE) nn_kernel<float, NN_UPDATE><<<g, NT, 0, s>>>(p);
    else if (mode == NN_ANALYSIS) nn_kernel<float, NN_ANALYSIS><<<g, NT, 0, s>>>(p);
    else nn_kernel<float, NN_RESIDUAL><<<g, NT, 0, s>>>(p);
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
