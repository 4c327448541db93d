// Small kernels of the blocked solve (gfx950):
//  - Step 1 as a row scaling, Y = R^{-1} X (eq. SM-step-1);
//  - the FP64 factorisation of one panel: with P = V_K^T [U_K, X] (b rows),
//    M = I + V_K^T U_K (symmetrised) = L D L^T by forward elimination, whose
//    pivots D are the gamma_k of the panel's b levels (Section 3.3); the
//    kernel leaves S = D^{-1/2} L^{-1} for the panel update
//    X <- X - U_K M^{-1} V_K^T X (eq. SWM with a rank-b term);
//  - Q = M^{-1} P_X = S^T (S P_X), two triangular products on the FP64
//    matrix cores.
#include <type_traits>

#include "enkf_internal.h"
#include "mfma_common.h"
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

// 1/x to within a few ulp: the hardware estimate refined by two Newton steps
// (each squares the relative error of the estimate).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

constexpr int PF_TI = 32, PF_TJ = 16;  // thread grid: rows x columns
constexpr int PF_NT = PF_TI * PF_TJ;    // 512 threads: 8 waves, two per SIMD

// One block of 512 threads as a 32 x 16 grid; thread (ti, tj) keeps the
// elements (i, j) = (ti + 32 r, tj + 16 c), r < 4, c < 8, of the symmetrised
// M = I + (P_K + P_K^T)/2 (padded with identity rows to a multiple of 4) in
// registers, and runs the forward elimination of [M | I] in place, four
// pivots at a time (no pivoting: M is SPD). A step on K = {k0..k0+3}, with
// A_KK = L4 D4 L4^T and W = A_KK^{-1}, takes every row i below K to
//   row_i <- row_i - (A_iK W) row_K,
// in the columns left of K (where the identity half has become L^{-1}) and
// right of K (the trailing Schur complement, which stays symmetric), stores
// -(A_iK W) in the columns of K (the identity half there), and takes the
// rows of K to L4^{-1} row_K left of K. The 4 x 4 diagonal block keeps D4 on
// its diagonal and L4^{-1} below it. When the sweeps are done the diagonal
// holds D of M = L D L^T, the pivots gamma_k of the panel's b levels
// (Section 3.3), and the strict lower triangle holds L^{-1}. Rows of K are
// published through the LDS (double-buffered: one barrier per four levels);
// by the symmetry of the trailing block, row K read at column i is also A_iK.
// Output: S = D^{-1/2} L^{-1} (lower triangular), so M^{-1} = S^T S, applied
// as two triangular products rather than through an explicit inverse of M,
// whose rounding grows with the condition of M.
__global__ __launch_bounds__(PF_NT) void panel_factor_kernel(int b, const double* __restrict__ P, int64_t ldp,
                                                             double* __restrict__ gamma_out, double* __restrict__ S,
                                                             unsigned* status) {
  constexpr int MP = kMaxPanel;
  constexpr int RR = MP / PF_TI, CC = MP / PF_TJ;  // rows and columns per thread
  constexpr int SUB = PF_TJ / 4;                   // four-pivot steps per column group
  static_assert(SUB % 2 == 0 && PF_TI % PF_TJ == 0, "buffers alternate within a group; a group's rows in one row group");
  __shared__ double pan[2][4 * MP];
  __shared__ double dsh[MP];
  const int t = threadIdx.x, ti = t % PF_TI, tj = t / PF_TI;
  const int b4 = (b + 3) / 4 * 4;
  double a[RR][CC];
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int i = ti + PF_TI * r, j = tj + PF_TJ * c;
      const int ic = min(i, b - 1), jc = min(j, b - 1);
      const double x = P[ic + (int64_t)jc * ldp], y = P[jc + (int64_t)ic * ldp];
      a[r][c] = (i < b && j < b) ? (i == j ? 1.0 : 0.0) + 0.5 * (x + y) : (i == j && i < b4 ? 1.0 : 0.0);
    }
  if (ti < 4)                                      // rows 0..3
#pragma unroll
    for (int c = 0; c < CC; ++c) pan[0][ti * MP + tj + PF_TJ * c] = a[0][c];
  __syncthreads();
  auto phase = [&](auto kb_c) {
    constexpr int KB = decltype(kb_c)::value;      // column group of the pivots
    constexpr int RK = KB * PF_TJ / PF_TI;         // row group of the pivots
    if (PF_TJ * KB >= b4) return;
#pragma unroll 1
    for (int ss = 0; ss < SUB; ++ss) {
      const int k0 = PF_TJ * KB + 4 * ss;
      if (k0 >= b4) break;
      const double* Pc = pan[ss & 1];              // rows k0..k0+3, every column
      double* Pn = pan[(ss + 1) & 1];
      // A_KK = L4 D4 L4^T and W = A_KK^{-1} = L4^{-T} D4^{-1} L4^{-1}
      double Lm[4][4], dv[4], iv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double e = Pc[q * MP + k0 + q];
#pragma unroll
        for (int u = 0; u < q; ++u) e -= Lm[q][u] * Lm[q][u] * dv[u];
        dv[q] = e;
        iv[q] = recip(e);
#pragma unroll
        for (int v = q + 1; v < 4; ++v) {
          double f = Pc[q * MP + k0 + v];
#pragma unroll
          for (int u = 0; u < q; ++u) f -= Lm[v][u] * Lm[q][u] * dv[u];
          Lm[v][q] = f * iv[q];
        }
      }
      double Li[4][4];                             // L4^{-1}, unit lower
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u > q) {
            Li[q][u] = 0.0;
          } else if (u == q) {
            Li[q][u] = 1.0;
          } else {
            double x = 0.0;
#pragma unroll
            for (int v = u; v < q; ++v) x -= Lm[q][v] * Li[v][u];
            Li[q][u] = x;
          }
        }
      double W[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double x = 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u) x += Li[u][q] * iv[u] * Li[u][v];
          W[q][v] = x;
        }
      if (t == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dsh[k0 + q] = dv[q];
          if (k0 + q < b) {
            gamma_out[k0 + q] = dv[q];
            if (!(dv[q] > 0.0) || !__builtin_isfinite(dv[q])) atomicOr(status, kStatusNotSpd);
          }
        }
      // rows below K: g_i = A_iK W (A_iK = row K at column i); other rows: 0,
      // so the uniform update below leaves them as they are
      double g[RR][4];
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        const int i = ti + PF_TI * r;
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = Pc[q * MP + i];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double y = fma(x[3], W[3][v], fma(x[2], W[2][v], fma(x[1], W[1][v], x[0] * W[0][v])));
          g[r][v] = i >= k0 + 4 ? y : 0.0;
        }
      }
      const int pi = ti - k0 % PF_TI, pj = tj - k0 % PF_TJ;
      const bool rowK = pi >= 0 && pi < 4, colK = pj >= 0 && pj < 4;
      // rows below K: A_ij -= g_i . A_Kj; rows of K, left of K: L4^{-1} row_K
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        double h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = Pc[q * MP + tj + PF_TJ * c];
#pragma unroll
        for (int r = 0; r < RR; ++r)
          a[r][c] = fma(-g[r][3], h[3], fma(-g[r][2], h[2], fma(-g[r][1], h[1], fma(-g[r][0], h[0], a[r][c]))));
        if (rowK && tj + PF_TJ * c < k0) {
          double x = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q == pi) x = ((Li[q][0] * h[0] + Li[q][1] * h[1]) + Li[q][2] * h[2]) + Li[q][3] * h[3];
          a[RK][c] = x;
        }
      }
      if (colK) {                                  // columns of K: -g_i below K; the K x K block: D4 and L4^{-1}
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          double x = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q == pj) x = -g[r][q];
          if (ti + PF_TI * r >= k0 + 4) a[r][KB] = x;
        }
        if (rowK) {
          double x = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (q == pi && v == pj) x = q > v ? Li[q][v] : (q == v ? dv[q] : 0.0);
          a[RK][KB] = x;
        }
      }
      // the next four rows
      const int kn = k0 + 4;
      const int pn = ti - kn % PF_TI;
      if (kn < b4 && pn >= 0 && pn < 4) {
        if (ss < SUB - 1) {
#pragma unroll
          for (int c = 0; c < CC; ++c) Pn[pn * MP + tj + PF_TJ * c] = a[RK][c];
        } else {
          if constexpr (KB < CC - 1) {
            constexpr int RN = (KB + 1) * PF_TJ / PF_TI;
#pragma unroll
            for (int c = 0; c < CC; ++c) Pn[pn * MP + tj + PF_TJ * c] = a[RN][c];
          }
        }
      }
      __syncthreads();
    }
  };
  phase(std::integral_constant<int, 0>{});
  phase(std::integral_constant<int, 1>{});
  phase(std::integral_constant<int, 2>{});
  phase(std::integral_constant<int, 3>{});
  phase(std::integral_constant<int, 4>{});
  phase(std::integral_constant<int, 5>{});
  phase(std::integral_constant<int, 6>{});
  phase(std::integral_constant<int, 7>{});
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int i = ti + PF_TI * r;
    if (i >= b) continue;
    const double rs = 1.0 / sqrt(dsh[i]);
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int j = tj + PF_TJ * c;
      if (j < b) S[i + (int64_t)j * b] = i > j ? a[r][c] * rs : (i == j ? rs : 0.0);
    }
  }
}

// Q = M^{-1} P_X = S^T (S P_X) on the FP64 matrix cores, S = D^{-1/2} L^{-1}
// lower triangular (b <= 128). Block = 32 columns of P (two 16-column
// tiles); wave w takes the 16-row tiles w and w + 4. First Y = S P_X (row
// tile i0 sums k < i0 + 16 only) into the LDS, then Q = S^T Y (row tile i0
// sums k >= i0 only). Indices past b or m are clamped, inner indices past b
// contribute zero.
__global__ __launch_bounds__(256) void tri_apply_kernel(int b, int m, const double* __restrict__ S,
                                                        const double* __restrict__ Pr, int64_t ldp,
                                                        double* __restrict__ Q) {
  __shared__ double Ysh[kMaxPanel][33];
  const int l = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int nt = (b + 15) / 16;
  int64_t jb[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) jb[c] = min(j0 + 16 * c + l % 16, (int64_t)m - 1);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int tr = w + 4 * tt;
    if (tr >= nt) continue;
    const int i0 = 16 * tr, ia = min(i0 + l % 16, b - 1);
    const int kend = min(b, i0 + 16);
    mf_d4 acc[2] = {MfmaF64::zero(), MfmaF64::zero()};
    for (int k = 0; k < kend; k += 4) {
      const int kk = k + l / 16, kc = min(kk, b - 1);
      const double av = kk < b ? S[ia + (int64_t)kc * b] : 0.0;
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[c] = MfmaF64::mma(av, Pr[kc + jb[c] * ldp], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) Ysh[i0 + MfmaF64::row(l, r)][16 * c + l % 16] = acc[c][r];
  }
  __syncthreads();
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int tr = w + 4 * tt;
    if (tr >= nt) continue;
    const int i0 = 16 * tr, ia = min(i0 + l % 16, b - 1);
    mf_d4 acc[2] = {MfmaF64::zero(), MfmaF64::zero()};
    for (int k = i0; k < b; k += 4) {
      const int kk = k + l / 16, kc = min(kk, b - 1);
      const double av = kk < b ? S[kc + (int64_t)ia * b] : 0.0;
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[c] = MfmaF64::mma(av, Ysh[kc][16 * c + l % 16], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + MfmaF64::row(l, r);
        const int64_t j = j0 + 16 * c + l % 16;
        if (i < b && j < m) Q[i + j * b] = acc[c][r];
      }
  }
}

// Y = X / scale in FP32 (scale = sqrt(sumsq / (n m)), the rms of what the
// sum of squares was taken over, when sumsq is given), so a shrinking
// residual stays inside the range of the narrow input types. With r, also
// Step 1 of the solve in the same pass: Y = R^{-1} X / scale, one rounding to
// FP32; latches NOT_SPD for r_i <= 0 or non-finite.
__global__ __launch_bounds__(256) void convert_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                      float* __restrict__ Y, int64_t ldy, const double* sumsq,
                                                      const double* __restrict__ r, unsigned* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double div = rms_scale(sumsq, (double)n * m);
  if (r) {
    const double rv = r[i];
    if (blockIdx.y == 0 && (!(rv > 0.0) || !__builtin_isfinite(rv))) atomicOr(status, kStatusNotSpd);
    div *= rv;
  }
  for (int j = blockIdx.y; j < m; j += gridDim.y) Y[i + (int64_t)j * ldy] = (float)(X[i + (int64_t)j * ldx] / div);
}

// Z += X (FP64), the correction of an FP64 refinement step.
__global__ __launch_bounds__(256) void add_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                  double* __restrict__ Z, int64_t ldz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = blockIdx.y; j < m; j += gridDim.y) Z[i + (int64_t)j * ldz] += X[i + (int64_t)j * ldx];
}

constexpr int NORM_BLOCKS = 1024;

// Per-block partial sums of squares of an n x m FP64 matrix, in a fixed
// order; then one block sums the partials.
__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                                                            const double* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t total = n * (int64_t)m;
  double sx = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % n, j = e / n;
    const double x = r ? X[i + j * ldx] / r[i] : X[i + j * ldx];
    sx += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) sx += __shfl_xor(sx, off, 64);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (lane == 0) red[w] = sx;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(64) void sumsq_final_kernel(int nblk, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  double sx = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) sx += part[b];
  for (int off = 32; off > 0; off >>= 1) sx += __shfl_xor(sx, off, 64);
  if (threadIdx.x == 0) out[0] = sx;
}

}  // namespace

int norm_partial_elems() { return NORM_BLOCKS; }

enkf_status launch_convert(int64_t n, int m, const double* X, int64_t ldx, float* Y, int64_t ldy, const double* sumsq,
                           const double* r, unsigned* status, hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  if (r && !status) return fail(ENKF_ERR_INVALID_ARG, "convert: row scaling needs the status word");
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(m < 16 ? m : 16));
  convert_kernel<<<grid, 256, 0, s>>>(n, m, X, ldx, Y, ldy, sumsq, r, status);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status launch_sumsq(int64_t n, int m, const double* X, int64_t ldx, const double* r, double* part, double* out,
                         hipStream_t s) {
  const int64_t total = n * (int64_t)m;
  int nblk = (int)((total + 255) / 256);
  if (nblk > NORM_BLOCKS) nblk = NORM_BLOCKS;
  if (nblk < 1) nblk = 1;
  sumsq_partial_kernel<<<nblk, 256, 0, s>>>(n, m, X, ldx, r, part);
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

enkf_status launch_panel_factor(int b, const double* P, int64_t ldp, double* gamma_out, double* S, unsigned* status,
                                hipStream_t s) {
  if (b < 1 || b > kMaxPanel) return fail(ENKF_ERR_NOT_SUPPORTED, "panel width outside [1, 128]");
  panel_factor_kernel<<<1, PF_NT, 0, s>>>(b, P, ldp, gamma_out, S, status);
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

enkf_status launch_panel_apply(int b, int m, const double* S, const double* Pr, int64_t ldp, double* Q,
                               hipStream_t s) {
  if (m <= 0) return ENKF_SUCCESS;
  if (b < 1 || b > kMaxPanel) return fail(ENKF_ERR_NOT_SUPPORTED, "panel width outside [1, 128]");
  const int64_t ct = ((int64_t)m + 31) / 32;
  if (ct > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "panel product: too many columns");
  tri_apply_kernel<<<(unsigned)ct, 256, 0, s>>>(b, m, S, Pr, ldp, Q);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
