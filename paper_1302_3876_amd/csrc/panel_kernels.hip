// Small kernels of the blocked solve (gfx950):
//  - Step 1 as a row scaling, Y = R^{-1} X (eq. SM-step-1);
//  - the FP64 factorisation of one panel: with P = V_K^T [U_K, X] (b rows),
//    M = I + V_K^T U_K (symmetrised) is inverted by symmetric sweeps whose
//    pivots are those of M = L D L^T, the gamma_k of the panel's b levels
//    (Section 3.3); the kernel leaves M^{-1} for the panel update
//    X <- X - U_K M^{-1} V_K^T X (eq. SWM with a rank-b term);
//  - Q = M^{-1} P_X, a b x m product in FP64.
#include "enkf_internal.h"
#include "panel.h"

namespace enkf {
namespace {


template <typename T>
__global__ __launch_bounds__(256) void scale_rows_kernel(int64_t n, int m, const T* __restrict__ X, int64_t ldx,
                                                         const double* __restrict__ r, T* __restrict__ Y, int64_t ldy,
                                                         unsigned* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const double rv = r[i];
  if (c == 0 && (!(rv > 0.0) || !__builtin_isfinite(rv))) atomicOr(status, kStatusNotSpd);
  for (int j = c; j < m; j += gridDim.y) Y[i + (int64_t)j * ldy] = (T)((double)X[i + (int64_t)j * ldx] / rv);
}

// One block of 256 threads as a 16 x 16 grid; thread (ti, tj) keeps the
// elements (i, j) = (ti + 16 r, tj + 16 c), r, c < 8, of the symmetrised
// M = I + (P_K + P_K^T)/2 in registers. M is inverted in place by b
// symmetric sweeps (Gauss-Jordan elimination in the natural order, without
// pivoting, which M being SPD allows): sweep k divides by the current
// diagonal element k, which is the k-th pivot of M = L D L^T, i.e. the
// gamma of level k0 + k. After the b sweeps the registers hold -M^{-1}.
// Only column k is shared per sweep (through LDS, double-buffered: one
// barrier per sweep).
__global__ __launch_bounds__(256) void panel_factor_kernel(int b, const double* __restrict__ P, int64_t ldp,
                                                           double* __restrict__ gamma_out, double* __restrict__ Minv,
                                                           unsigned* status) {
  __shared__ double col[2][kMaxPanel];
  const int t = threadIdx.x, ti = t % 16, tj = t / 16;
  double a[8][8];
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = ti + 16 * r, j = tj + 16 * c;
      const int ic = min(i, b - 1), jc = min(j, b - 1);
      const double x = P[ic + (int64_t)jc * ldp], y = P[jc + (int64_t)ic * ldp];
      a[r][c] = (i < b && j < b) ? (i == j ? 1.0 : 0.0) + 0.5 * (x + y) : 0.0;
    }
  if (tj == 0)
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (ti + 16 * r < b) col[0][ti + 16 * r] = a[r][0];
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    const double* __restrict__ ck = col[k & 1];
    double* __restrict__ cn = col[(k + 1) & 1];
    const double d = ck[k];
    if (t == 0) {
      gamma_out[k] = d;
      if (!(d > 0.0) || !__builtin_isfinite(d)) atomicOr(status, kStatusNotSpd);
    }
    const double inv = 1.0 / d;
    double ci[8], cj[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) ci[r] = ck[min(ti + 16 * r, b - 1)];
#pragma unroll
    for (int c = 0; c < 8; ++c) cj[c] = ck[min(tj + 16 * c, b - 1)];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int i = ti + 16 * r, j = tj + 16 * c;
        // by symmetry, element (k, j) of the current matrix is ck[j]
        const double upd = a[r][c] - ci[r] * cj[c] * inv;
        double v = upd;
        if (i == k) v = cj[c] * inv;
        if (j == k) v = ci[r] * inv;
        if (i == k && j == k) v = -inv;
        a[r][c] = v;
        if (j == k + 1 && i < b) cn[i] = v;
      }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = ti + 16 * r, j = tj + 16 * c;
      if (i < b && j < b) Minv[i + (int64_t)j * b] = -a[r][c];
    }
}

__global__ __launch_bounds__(256) void small_gemm_kernel(int b, int m, const double* __restrict__ Minv,
                                                         const double* __restrict__ Pr, int64_t ldp,
                                                         double* __restrict__ Q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)b * m) return;
  const int i = (int)(e % b);
  const int64_t j = e / b;
  double s = 0.0;
  for (int k = 0; k < b; ++k) s += Minv[i + (int64_t)k * b] * Pr[k + j * ldp];
  Q[i + j * b] = s;
}

// Scale of a residual block: its root mean square (1 when it is zero or
// when no sum of squares is given).
__device__ __forceinline__ double rms_scale(const double* sumsq, double count) {
  if (!sumsq) return 1.0;
  const double s = sqrt(sumsq[0] / count);
  return (s > 0.0 && s < 1e300) ? s : 1.0;
}

// Y = X / scale in FP32 (scale = rms of X when sumsq is given), so a
// shrinking residual stays inside the range of the narrow input types.
__global__ __launch_bounds__(256) void convert_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                      float* __restrict__ Y, int64_t ldy, const double* sumsq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double inv = 1.0 / rms_scale(sumsq, (double)n * m);
  for (int j = blockIdx.y; j < m; j += gridDim.y) Y[i + (int64_t)j * ldy] = (float)(X[i + (int64_t)j * ldx] * inv);
}

// Z = scale W (accumulate == 0) or Z += scale W (accumulate == 1), W in FP32.
__global__ __launch_bounds__(256) void widen_kernel(int64_t n, int m, const float* __restrict__ W, int64_t ldw,
                                                    double* __restrict__ Z, int64_t ldz, int accumulate,
                                                    const double* sumsq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = rms_scale(sumsq, (double)n * m);
  for (int j = blockIdx.y; j < m; j += gridDim.y) {
    const double w = sc * (double)W[i + (int64_t)j * ldw];
    double* z = Z + i + (int64_t)j * ldz;
    *z = accumulate ? *z + w : w;
  }
}

// Z += X (FP64), the correction of an FP64 refinement step.
__global__ __launch_bounds__(256) void add_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                  double* __restrict__ Z, int64_t ldz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = blockIdx.y; j < m; j += gridDim.y) Z[i + (int64_t)j * ldz] += X[i + (int64_t)j * ldx];
}

constexpr int NORM_BLOCKS = 1024;

// Per-block partial sums of squares of two n x m FP64 matrices, in a fixed
// order; then one block sums the partials.
__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                            const double* __restrict__ Y, int64_t ldy,
                                                            double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t total = n * (int64_t)m;
  double sx = 0.0, sy = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % n, j = e / n;
    const double x = X[i + j * ldx], y = Y[i + j * ldy];
    sx += x * x;
    sy += y * y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off, 64);
    sy += __shfl_xor(sy, off, 64);
  }
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (lane == 0) { red[0][w] = sx; red[1][w] = sy; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    part[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

__global__ __launch_bounds__(64) void sumsq_final_kernel(int nblk, const double* __restrict__ part, double* __restrict__ out) {
  double sx = 0.0, sy = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) { sx += part[2 * b]; sy += part[2 * b + 1]; }
  for (int off = 32; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off, 64);
    sy += __shfl_xor(sy, off, 64);
  }
  if (threadIdx.x == 0) { out[0] = sx; out[1] = sy; }
}

}  // namespace

int norm_partial_elems() { return 2 * NORM_BLOCKS; }

enkf_status launch_convert(int64_t n, int m, const double* X, int64_t ldx, float* Y, int64_t ldy, const double* sumsq,
                           hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(m < 16 ? m : 16));
  convert_kernel<<<grid, 256, 0, s>>>(n, m, X, ldx, Y, ldy, sumsq);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_widen(int64_t n, int m, const float* W, int64_t ldw, double* Z, int64_t ldz, bool accumulate,
                         const double* sumsq, hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(m < 16 ? m : 16));
  widen_kernel<<<grid, 256, 0, s>>>(n, m, W, ldw, Z, ldz, accumulate ? 1 : 0, sumsq);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_sumsq2(int64_t n, int m, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* part,
                          double* out, hipStream_t s) {
  const int64_t total = n * (int64_t)m;
  int nblk = (int)((total + 255) / 256);
  if (nblk > NORM_BLOCKS) nblk = NORM_BLOCKS;
  if (nblk < 1) nblk = 1;
  sumsq_partial_kernel<<<nblk, 256, 0, s>>>(n, m, X, ldx, Y, ldy, part);
  ENKF_HIP_CHECK(hipGetLastError());
  sumsq_final_kernel<<<1, 64, 0, s>>>(nblk, part, out);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_scale_rows(enkf_dtype dt, int64_t n, int m, const void* X, int64_t ldx, const double* r, void* Y,
                              int64_t ldy, unsigned* status, hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(m < 16 ? m : 16));
  if (dt == ENKF_F64)
    scale_rows_kernel<double><<<grid, 256, 0, s>>>(n, m, (const double*)X, ldx, r, (double*)Y, ldy, status);
  else
    scale_rows_kernel<float><<<grid, 256, 0, s>>>(n, m, (const float*)X, ldx, r, (float*)Y, ldy, status);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_panel_factor(int b, const double* P, int64_t ldp, double* gamma_out, double* Minv, unsigned* status,
                                hipStream_t s) {
  if (b < 1 || b > kMaxPanel) return fail(ENKF_ERR_NOT_SUPPORTED, "panel width outside [1, 128]");
  panel_factor_kernel<<<1, 256, 0, s>>>(b, P, ldp, gamma_out, Minv, status);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_add(int64_t n, int m, const double* X, int64_t ldx, double* Z, int64_t ldz, hipStream_t s) {
  if (n <= 0 || m <= 0) return ENKF_SUCCESS;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(m < 16 ? m : 16));
  add_kernel<<<grid, 256, 0, s>>>(n, m, X, ldx, Z, ldz);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_small_gemm(int b, int m, const double* Minv, const double* Pr, int64_t ldp, double* Q,
                              hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  const int64_t total = (int64_t)b * m;
  small_gemm_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(b, m, Minv, Pr, ldp, Q);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
