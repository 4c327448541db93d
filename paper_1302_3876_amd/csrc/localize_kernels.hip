// Partial localization of the analysis update (Section 3.1.2, eq.
// localized-correction-component), for gfx950:
//   X^A[i, l] = X^B[i, l] + sum_j delta(i, j) (S V^T)[i, j] Z[j, l],
//   S = (X^B - xbar 1^T)/sqrt(N-1),
//   delta(i, j) = exp(-d(i, loc_j)/length), 0 past the radius (if any),
//   d the index distance, taken on a ring when ring > 0.
// The n_state x n_obs influence-weighted matrix is never formed in memory:
// a block owns 64 state rows and 128 columns of the correction and walks the
// observations 32 at a time; per step it forms the 64 x 32 tile of S V^T on
// the matrix cores (inner dimension N, in stages of KC), weights it with the
// impact factors computed in registers, stages it in LDS, and accumulates the
// tile times the 32 x 128 slice of Z on the matrix cores. 4 waves; the tile
// of S V^T is split by state rows (16 per wave), the correction by columns
// (32 per wave). With N > 128 the column chunks of a row tile recompute the
// S V^T tiles.
#include "enkf_internal.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int LZ_NT = 256;
constexpr int LZ_TI = 64;    // state rows per block
constexpr int LZ_TJ = 32;    // observations per step
constexpr int LZ_NC = 128;   // correction columns per block

template <typename T> struct LzMf;
template <> struct LzMf<double> { typedef MfmaF64 type; static constexpr int KC = 16; };
template <> struct LzMf<float> { typedef MfmaF32 type; static constexpr int KC = 32; };

template <typename T>
__global__ __launch_bounds__(LZ_NT) void localize_kernel(LocalizeArgs p) {
  typedef typename LzMf<T>::type MF;
  constexpr int KC = LzMf<T>::KC;
  constexpr int LDS_ROW = LZ_TI + 16;   // [k][state row] stages
  constexpr int LDV = LZ_TJ + 16;       // [k][obs]
  constexpr int LDZ = LZ_NC + 16;       // [obs][column]
  __shared__ T Ss[KC * LDS_ROW];
  __shared__ T Vs[KC * LDV];
  __shared__ T As[LZ_TJ * LDS_ROW];     // [obs][state row], weighted
  __shared__ T Zs[LZ_TJ * LDZ];
  __shared__ double mean[LZ_TI];
  __shared__ int64_t locs[LZ_TJ];
  const T* __restrict__ XB = static_cast<const T*>(p.XB);
  const T* __restrict__ V = static_cast<const T*>(p.V);
  const T* __restrict__ Z = static_cast<const T*>(p.Z);
  T* __restrict__ XA = static_cast<T*>(p.XA);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int64_t row0 = (int64_t)blockIdx.x * LZ_TI;
  const int c0 = blockIdx.y * LZ_NC;
  const int N = p.N;
  const int64_t ns = p.n_state, no = p.n_obs;

  {  // row means (fixed order: NT/TI partial sums per row, then in order)
    constexpr int Q = LZ_NT / LZ_TI;
    __shared__ double part[Q][LZ_TI];
    const int rr = t % LZ_TI, q = t / LZ_TI;
    const T* __restrict__ xr = XB + min(row0 + rr, ns - 1);
    double s = 0.0;
    for (int k = q; k < N; k += Q) s += (double)xr[(int64_t)k * p.ldx];
    part[q][rr] = s;
    __syncthreads();
    if (t < LZ_TI) {
      double tot = 0.0;
#pragma unroll
      for (int z = 0; z < Q; ++z) tot += part[z][t];
      mean[t] = tot / (double)N;
    }
    __syncthreads();
  }
  const double sinv = 1.0 / sqrt((double)(N - 1));

  typename MF::acc_t acc2[2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc2[c][rt] = MF::zero();

  for (int64_t j0 = 0; j0 < no; j0 += LZ_TJ) {
    // ---- phase 1: A = S V^T on rows [row0, +64) x obs [j0, +32)
    typename MF::acc_t acc1[2] = {MF::zero(), MF::zero()};
    if (t < LZ_TJ) locs[t] = p.loc[min(j0 + t, no - 1)];
    for (int k0 = 0; k0 < N; k0 += KC) {
      __syncthreads();
      for (int e = t; e < KC * LZ_TI; e += LZ_NT) {      // S stage [k][row], rows contiguous in X^B
        const int rr = e % LZ_TI, kk = e / LZ_TI;
        const int k = k0 + kk;
        const double x = (double)XB[min(row0 + rr, ns - 1) + (int64_t)min(k, N - 1) * p.ldx];
        Ss[kk * LDS_ROW + rr] = (T)(k < N ? (x - mean[rr]) * sinv : 0.0);
      }
      for (int e = t; e < KC * LZ_TJ; e += LZ_NT) {      // V stage [k][obs]
        const int jj = e % LZ_TJ, kk = e / LZ_TJ;
        const int k = k0 + kk;
        const T v = V[min(j0 + jj, no - 1) + (int64_t)min(k, N - 1) * p.ldv];
        Vs[kk * LDV + jj] = (k < N) ? v : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; kk += MF::KSTEP) {
        const T sop = Ss[(kk + l / 16) * LDS_ROW + 16 * w + l % 16];
#pragma unroll
        for (int c = 0; c < 2; ++c) acc1[c] = MF::mma(Vs[(kk + l / 16) * LDV + 16 * c + l % 16], sop, acc1[c]);
      }
    }
    // weight by the impact factors (zero past the last observation) and stage
    // as [obs][state row]
    const int64_t i = row0 + 16 * w + l % 16;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jj = 16 * c + MF::row(l, r);
        int64_t d = i - locs[jj];
        d = d < 0 ? -d : d;
        if (p.ring > 0 && p.ring - d < d) d = p.ring - d;
        double delta = exp(-(double)d / p.length);
        if ((p.radius >= 0 && d > p.radius) || j0 + jj >= no) delta = 0.0;
        As[jj * LDS_ROW + 16 * w + l % 16] = (T)(delta * (double)acc1[c][r]);
      }
    // Z slice [obs][column]
    for (int e = t; e < LZ_TJ * LZ_NC; e += LZ_NT) {
      const int jj = e % LZ_TJ, cc = e / LZ_TJ;
      const T z = Z[min(j0 + jj, no - 1) + (int64_t)min(c0 + cc, N - 1) * p.ldz];
      Zs[jj * LDZ + cc] = (j0 + jj < no) ? z : T(0);
    }
    __syncthreads();
    // ---- phase 2: correction += A Z
#pragma unroll
    for (int kk = 0; kk < LZ_TJ; kk += MF::KSTEP) {
      T zop[2], aop[4];
#pragma unroll
      for (int c = 0; c < 2; ++c) zop[c] = Zs[(kk + l / 16) * LDZ + 32 * w + 16 * c + l % 16];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) aop[rt] = As[(kk + l / 16) * LDS_ROW + 16 * rt + l % 16];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc2[c][rt] = MF::mma(zop[c], aop[rt], acc2[c][rt]);
    }
  }
  // X^A = X^B + correction; acc2[c][rt] element: column (row of the result),
  // state row (column of the result)
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = c0 + 32 * w + 16 * c + MF::row(l, r);
        const int64_t i = row0 + 16 * rt + l % 16;
        if (col < N && i < ns) {
          const double xb = (double)XB[i + (int64_t)col * p.ldx];
          XA[i + (int64_t)col * p.ldxa] = (T)(xb + (double)acc2[c][rt][r]);
        }
      }
}

}  // namespace

enkf_status launch_localize(enkf_dtype dt, const LocalizeArgs& a, hipStream_t s) {
  if (a.n_state <= 0 || a.N <= 0) return ENKF_SUCCESS;
  const int64_t rt = (a.n_state + LZ_TI - 1) / LZ_TI;
  const int ct = (a.N + LZ_NC - 1) / LZ_NC;
  if (rt > 0x7fffffff || ct > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "localized analysis: grid too large");
  dim3 grid((unsigned)rt, (unsigned)ct);
  if (dt == ENKF_F64) localize_kernel<double><<<grid, LZ_NT, 0, s>>>(a);
  else localize_kernel<float><<<grid, LZ_NT, 0, s>>>(a);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
