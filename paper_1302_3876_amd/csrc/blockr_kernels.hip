// Step 1 with a block-diagonal R (Section 2.1: R = diag(R_1, ..., R_B),
// each R_b SPD of size N_b; Section 3.1: Z0 = R^{-1} D and U0 = R^{-1} V,
// which cost O(n N^2) at most, Section 3.2), for gfx950.
//   - chol_kernel: one wave per block, R_b = L L^T in LDS (FP64, right-
//     looking), L stored packed like the blocks; a pivot that is not > 0 or
//     not finite latches the not-SPD status;
//   - block_solve_kernel: one thread per (block, column): L y = x, L^T z = y
//     in FP64 registers (blocks of up to S rows, S a compile-time bound), in
//     place allowed. Consecutive threads take consecutive blocks of the same
//     column, so the column reads are contiguous across the wave.
#include "enkf_internal.h"

namespace enkf {
namespace {

constexpr int BR_MAX = kMaxRBlock;

__global__ __launch_bounds__(64) void chol_kernel(const int64_t* __restrict__ off, const int64_t* __restrict__ poff,
                                                  const double* __restrict__ Rb, double* __restrict__ Lf,
                                                  unsigned* status) {
  __shared__ double A[BR_MAX][BR_MAX + 1];
  const int64_t b = blockIdx.x;
  const int s = (int)(off[b + 1] - off[b]);
  const double* __restrict__ src = Rb + poff[b];
  const int t = threadIdx.x;
  for (int e = t; e < s * s; e += 64) A[e % s][e / s] = src[e];
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    const double d = A[j][j];
    if (t == 0 && (!(d > 0.0) || !__builtin_isfinite(d))) atomicOr(status, kStatusNotSpd);
    const double ljj = sqrt(d);
    __syncthreads();
    if (t > j && t < s) A[t][j] /= ljj;
    if (t == j) A[j][j] = ljj;
    __syncthreads();
    if (t > j && t < s) {
      const double lij = A[t][j];
      for (int k = j + 1; k <= t; ++k) A[t][k] -= lij * A[k][j];
    }
    __syncthreads();
  }
  double* __restrict__ dst = Lf + poff[b];
  for (int e = t; e < s * s; e += 64) {
    const int i = e % s, k = e / s;
    dst[e] = i >= k ? A[i][k] : 0.0;
  }
}

template <typename T, int S>
__global__ __launch_bounds__(256) void block_solve_kernel(int64_t nblk, int m, const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ poff,
                                                          const double* __restrict__ Lf, const T* X, int64_t ldx,
                                                          T* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nblk * m) return;
  const int64_t b = e % nblk;
  const int c = (int)(e / nblk);
  const int64_t r0 = off[b];
  const int s = (int)(off[b + 1] - r0);
  const double* __restrict__ L = Lf + poff[b];
  const T* x = X + r0 + (int64_t)c * ldx;
  T* y = Y + r0 + (int64_t)c * ldy;
  double v[S];
#pragma unroll
  for (int i = 0; i < S; ++i) v[i] = i < s ? (double)x[i] : 0.0;
  // L w = x (forward), column-oriented: w_i final once reached
#pragma unroll
  for (int i = 0; i < S; ++i) {
    if (i < s) {
      const double wi = v[i] / L[i + i * s];
      v[i] = wi;
#pragma unroll
      for (int k = i + 1; k < S; ++k)
        if (k < s) v[k] -= L[k + i * s] * wi;
    }
  }
  // L^T z = w (backward)
#pragma unroll
  for (int i = S - 1; i >= 0; --i) {
    if (i < s) {
      double zi = v[i];
#pragma unroll
      for (int k = i + 1; k < S; ++k)
        if (k < s) zi -= L[k + i * s] * v[k];
      v[i] = zi / L[i + i * s];
    }
  }
#pragma unroll
  for (int i = 0; i < S; ++i)
    if (i < s) y[i] = (T)v[i];
}

template <typename T, int S>
void solve_go(int64_t nblk, int m, const int64_t* off, const int64_t* poff, const double* Lf, const void* X,
              int64_t ldx, void* Y, int64_t ldy, hipStream_t st) {
  const int64_t total = nblk * m;
  block_solve_kernel<T, S><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(
      nblk, m, off, poff, Lf, static_cast<const T*>(X), ldx, static_cast<T*>(Y), ldy);
}

template <typename T>
void solve_pick(int max_bs, int64_t nblk, int m, const int64_t* off, const int64_t* poff, const double* Lf,
                const void* X, int64_t ldx, void* Y, int64_t ldy, hipStream_t st) {
  if (max_bs <= 4) solve_go<T, 4>(nblk, m, off, poff, Lf, X, ldx, Y, ldy, st);
  else if (max_bs <= 8) solve_go<T, 8>(nblk, m, off, poff, Lf, X, ldx, Y, ldy, st);
  else if (max_bs <= 16) solve_go<T, 16>(nblk, m, off, poff, Lf, X, ldx, Y, ldy, st);
  else if (max_bs <= 32) solve_go<T, 32>(nblk, m, off, poff, Lf, X, ldx, Y, ldy, st);
  else solve_go<T, 64>(nblk, m, off, poff, Lf, X, ldx, Y, ldy, st);
}

}  // namespace

enkf_status launch_block_chol(int64_t nblk, const int64_t* off, const int64_t* poff, const double* Rb, double* Lf,
                              unsigned* status, hipStream_t s) {
  if (nblk > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "block R: too many blocks");
  chol_kernel<<<(unsigned)nblk, 64, 0, s>>>(off, poff, Rb, Lf, status);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_block_solve(enkf_dtype dt, int max_bs, int64_t nblk, int m, const int64_t* off,
                               const int64_t* poff, const double* Lf, const void* X, int64_t ldx, void* Y, int64_t ldy,
                               hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  if (nblk * m / 256 > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "block R: grid too large");
  if (dt == ENKF_F64) solve_pick<double>(max_bs, nblk, m, off, poff, Lf, X, ldx, Y, ldy, s);
  else solve_pick<float>(max_bs, nblk, m, off, poff, Lf, X, ldx, Y, ldy, s);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
