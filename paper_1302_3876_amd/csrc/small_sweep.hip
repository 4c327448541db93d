// The plain iterative Sherman-Morrison factorisation and solve of a small
// FP64 system in one launch (Section 3.1, Steps 1-2), for gfx950.
#include "enkf_internal.h"

namespace enkf {
namespace {

// Small systems in FP64: Step 1 and all N levels in one block (8 waves),
// with the r-scaled columns and V resident in the LDS (n (2N + nrhs)
// doubles; a level costs one block barrier instead of a launch). Level k:
// every wave forms gamma_k = 1 + v_k^T u_k^{(k-1)} (factorisation; a solve
// reads it) and h_k = u_k / gamma_k; then wave w takes every eighth active
// column (U columns past k, then every Z column), four at a time:
// c_q = v_k^T x_q (lanes over rows, a fixed-order wave reduction),
// x_q -= h_k c_q (eq. SM-step-2). A solve with a stored factor (Uin) takes
// u_k and gamma_k from it and updates only the Z columns with the same
// operations as the factorisation + solve, so both give bitwise the same Z.
// U (column k at its level) and Z are written at the end.
constexpr int kSmallThreads = 512;
__global__ __launch_bounds__(kSmallThreads) void small_sweep_kernel(SmallSweepArgs a) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  __shared__ double hs[kSmallSweepMaxRows];            // h_k = u_k / gamma_k
  const int64_t n = a.n;
  const bool solve_only = a.Uin != nullptr;
  const int N = a.N, nu = solve_only ? 0 : a.N, mt = nu + a.nrhs;   // columns of Xs: [U, Z] or [Z]
  double* Xs = sm;                                // [mt][n]
  double* Vs = sm + (size_t)mt * n;               // [N][n]
  double* Us = Vs + (size_t)N * n;                // [N][n], solves with a stored factor
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int nwave = (int)(blockDim.x / kWave);
  for (int64_t e = t; e < (int64_t)mt * n; e += blockDim.x) {
    const int64_t i = e % n;
    const int q = (int)(e / n);
    const double ri = a.r[i];
    if (q == 0 && (!(ri > 0.0) || !__builtin_isfinite(ri))) atomicOr(a.status, kStatusNotSpd);
    const double src = q < nu ? a.V[i + (int64_t)q * a.ldv] : a.D[i + (int64_t)(q - nu) * a.ldd];
    Xs[e] = src / ri;                             // Step 1 (eq. SM-step-1)
  }
  for (int64_t e = t; e < (int64_t)N * n; e += blockDim.x) {
    const int64_t i = e % n;
    const int q = (int)(e / n);
    Vs[e] = a.V[i + (int64_t)q * a.ldv];
    if (solve_only) Us[e] = a.Uin[i + (int64_t)q * a.ldu];
  }
  __syncthreads();
  auto wred = [](double x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
  };
  constexpr int CB = 4;                           // columns per wave reduced together
  for (int k = 0; k < N; ++k) {
    const double* vk = Vs + (size_t)k * n;
    const double* uk = solve_only ? Us + (size_t)k * n : Xs + (size_t)k * n;
    // gamma_k and h_k = u_k / gamma_k: every wave forms the same values from
    // the same LDS data and stores them (bitwise equal stores to the same
    // words), so no barrier is needed before the columns; the barrier that
    // ends each level keeps level k + 1's stores after every read of level k
    double* h = hs;
    {
      double g;
      if (solve_only) {
        g = a.gamma[k];
      } else {
        double sacc = 0.0;
        for (int64_t i = l; i < n; i += kWave) sacc = fma(vk[i], uk[i], sacc);
        g = 1.0 + wred(sacc);
        if (w == 0 && l == 0) {
          a.gamma[k] = g;
          if (!(g > 0.0) || !__builtin_isfinite(g)) atomicOr(a.status, kStatusNotSpd);
        }
      }
      for (int64_t i = l; i < n; i += kWave) h[i] = uk[i] / g;
    }
    // active columns: U columns k+1 .. N-1, then the Z columns; wave w takes
    // every nwave-th one, CB at a time (a column's result does not depend on
    // which wave takes it or with which others)
    const int q0 = solve_only ? 0 : k + 1, na = mt - q0;
    for (int j0 = w; j0 < na; j0 += CB * nwave) {
      double c[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int j = j0 + u * nwave;
        double acc = 0.0;
        if (j < na) {
          const double* xq = Xs + (size_t)(q0 + j) * n;
          for (int64_t i = l; i < n; i += kWave) acc = fma(vk[i], xq[i], acc);
        }
        c[u] = acc;
      }
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
        for (int u = 0; u < CB; ++u) c[u] += __shfl_xor(c[u], off, kWave);
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int j = j0 + u * nwave;
        if (j < na) {
          double* xq = Xs + (size_t)(q0 + j) * n;
          for (int64_t i = l; i < n; i += kWave) xq[i] -= h[i] * c[u];
        }
      }
    }
    __syncthreads();
  }
  for (int64_t e = t; e < (int64_t)mt * n; e += blockDim.x) {
    const int64_t i = e % n;
    const int q = (int)(e / n);
    if (q < nu) a.U[i + (int64_t)q * a.ldu] = Xs[e];
    else a.Z[i + (int64_t)(q - nu) * a.ldz] = Xs[e];
  }
}

}  // namespace

size_t small_sweep_lds_bytes(int64_t n, int N, int nrhs) {
  return sizeof(double) * (size_t)n * (size_t)(2 * N + nrhs);
}

enkf_status launch_small_sweep(const SmallSweepArgs& a, hipStream_t s) {
  const size_t bytes = small_sweep_lds_bytes(a.n, a.N, a.nrhs);
  if (a.n < 1 || a.n > kSmallSweepMaxRows || a.N < 1 || a.nrhs < 0 || bytes > kSmallSweepMaxLds)
    return fail(ENKF_ERR_INVALID_ARG, "small sweep: the system does not fit the LDS");
  small_sweep_kernel<<<1, kSmallThreads, bytes, s>>>(a);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
