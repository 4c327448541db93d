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
// S V^T tiles. Ensembles of at most 64 members take a specialised kernel
// (localize64_kernel) that keeps the S tile resident.
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

// Two waves per SIMD at least (the LDS allows no more): the accumulators then
// stay in VGPRs instead of being split off into accumulation registers.
template <typename T>
__global__ __launch_bounds__(LZ_NT, 2) void localize_kernel(LocalizeArgs p) {
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

// N <= 64 (padded to 64): the block's 64 x 64 tile of S stays in the LDS for
// the whole walk over the observations; each step loads the 32 observations'
// 64 x 32 slice of V^T and 32 x 64 slice of Z into registers one step ahead
// (branch-free: indices past the data are clamped and the values zeroed when
// staged), forms the 64 x 32 tile of S V^T (wave w: state rows 16w..16w+15),
// weights it and accumulates it times the Z slice (wave w: columns
// 16w..16w+15). The weighted tile takes the place of the V slice in the LDS.
constexpr int L6_TI = 64;    // state rows per block
constexpr int L6_TJ = 32;    // observations per step
constexpr int L6_K = 64;     // members, padded

template <typename T>
__global__ __launch_bounds__(LZ_NT, sizeof(T) == 8 ? 2 : 3) void localize64_kernel(LocalizeArgs p) {
  typedef typename LzMf<T>::type MF;
  constexpr int PAD = sizeof(T) == 8 ? 8 : 16;
  constexpr int LDS_ = L6_TI + PAD;     // Ss[k][state row]
  constexpr int LDV = L6_TJ + PAD;      // Vs[k][obs]
  constexpr int LDA = L6_TI + PAD;      // As[obs][state row] (aliases Vs)
  constexpr int LDZ = L6_K + PAD;       // Zs[obs][column]
  constexpr int VA = L6_K * LDV > L6_TJ * LDA ? L6_K * LDV : L6_TJ * LDA;
  constexpr int PV = L6_TJ * L6_K / LZ_NT;   // staged V (and Z) elements per thread
  __shared__ T Ss[L6_K * LDS_];
  __shared__ T VAs[VA];
  __shared__ T Zs[L6_TJ * LDZ];
  __shared__ double mean[L6_TI];
  __shared__ int64_t locs[L6_TJ];
  T* Vs = VAs;
  T* As = VAs;
  const T* __restrict__ XB = static_cast<const T*>(p.XB);
  const T* __restrict__ V = static_cast<const T*>(p.V);
  const T* __restrict__ Z = static_cast<const T*>(p.Z);
  T* __restrict__ XA = static_cast<T*>(p.XA);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int64_t row0 = (int64_t)blockIdx.x * L6_TI;
  const int N = p.N;
  const int64_t ns = p.n_state, no = p.n_obs;

  {  // row means (fixed order: NT/TI partial sums per row, then in order)
    constexpr int Q = LZ_NT / L6_TI;
    __shared__ double part[Q][L6_TI];
    const int rr = t % L6_TI, q = t / L6_TI;
    const T* __restrict__ xr = XB + min(row0 + rr, ns - 1);
    double sum = 0.0;
    for (int k = q; k < N; k += Q) sum += (double)xr[(int64_t)k * p.ldx];
    part[q][rr] = sum;
    __syncthreads();
    if (t < L6_TI) {
      double tot = 0.0;
#pragma unroll
      for (int z = 0; z < Q; ++z) tot += part[z][t];
      mean[t] = tot / (double)N;
    }
    __syncthreads();
  }
  {  // the S tile, once
    const double sinv = 1.0 / sqrt((double)(N - 1));
    const int rr = t % L6_TI;
    const T* __restrict__ xr = XB + min(row0 + rr, ns - 1);
    for (int k = t / L6_TI; k < L6_K; k += LZ_NT / L6_TI) {
      const double x = (double)xr[(int64_t)min(k, N - 1) * p.ldx];
      Ss[k * LDS_ + rr] = (T)(k < N ? (x - mean[rr]) * sinv : 0.0);
    }
  }
  // staged slices: thread (obs jj = t % 32, members / columns t / 32 + 8 q)
  const int jj = t % L6_TJ, kq = t / L6_TJ;
  const float inv_len = (float)(1.0 / p.length);
  T vreg[PV], zreg[PV];
  int64_t lreg = 0;
  auto fetch = [&](int64_t j0) {
    const int64_t j = min(j0 + jj, no - 1);
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int64_t k = min(kq + 8 * q, N - 1);
      vreg[q] = V[j + k * p.ldv];
      zreg[q] = Z[j + k * p.ldz];
    }
    if (t < L6_TJ) lreg = p.loc[min(j0 + t, no - 1)];
  };
  typename MF::acc_t acc2[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc2[rt] = MF::zero();
  fetch(0);
  for (int64_t j0 = 0; j0 < no; j0 += L6_TJ) {
    __syncthreads();                              // the previous step is done with the LDS
    {
      const bool jok = j0 + jj < no;
#pragma unroll
      for (int q = 0; q < PV; ++q) {
        const int k = kq + 8 * q;
        const bool ok = jok && k < N;
        Vs[k * LDV + jj] = ok ? vreg[q] : T(0);
        Zs[jj * LDZ + k] = ok ? zreg[q] : T(0);
      }
      if (t < L6_TJ) locs[t] = lreg;
    }
    __syncthreads();
    fetch(j0 + L6_TJ);                            // past the end: clamped, unused
    __builtin_amdgcn_sched_barrier(0);
    // A = S V^T on state rows 16w.. x the step's 32 observations
    typename MF::acc_t acc1[2] = {MF::zero(), MF::zero()};
#pragma unroll
    for (int k = 0; k < L6_K; k += MF::KSTEP) {
      const T sop = Ss[(k + l / 16) * LDS_ + 16 * w + l % 16];
#pragma unroll
      for (int c = 0; c < 2; ++c) acc1[c] = MF::mma(Vs[(k + l / 16) * LDV + 16 * c + l % 16], sop, acc1[c]);
    }
    // impact factors (zero past the last observation or the radius)
    T wv[2][4];
    const int64_t i = row0 + 16 * w + l % 16;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jo = 16 * c + MF::row(l, r);
        int64_t d = i - locs[jo];
        d = d < 0 ? -d : d;
        if (p.ring > 0 && p.ring - d < d) d = p.ring - d;
        // the factor in the storage precision (FP32 storage: expf)
        T delta;
        if constexpr (sizeof(T) == 8) delta = exp(-(double)d / p.length);
        else delta = expf(-(float)d * inv_len);
        if ((p.radius >= 0 && d > p.radius) || j0 + jo >= no) delta = T(0);
        wv[c][r] = delta * acc1[c][r];
      }
    __syncthreads();                              // every wave is done with Vs
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) As[(16 * c + MF::row(l, r)) * LDA + 16 * w + l % 16] = wv[c][r];
    __syncthreads();
    // correction += A Z on columns 16w..16w+15
#pragma unroll
    for (int kk = 0; kk < L6_TJ; kk += MF::KSTEP) {
      const T zop = Zs[(kk + l / 16) * LDZ + 16 * w + l % 16];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) acc2[rt] = MF::mma(zop, As[(kk + l / 16) * LDA + 16 * rt + l % 16], acc2[rt]);
    }
  }
  // X^A = X^B + correction; acc2[rt] element: column (row of the result),
  // state row (column of the result)
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = 16 * w + MF::row(l, r);
      const int64_t i = row0 + 16 * rt + l % 16;
      if (col < N && i < ns) {
        const double xb = (double)XB[i + (int64_t)col * p.ldx];
        XA[i + (int64_t)col * p.ldxa] = (T)(xb + (double)acc2[rt][r]);
      }
    }
}

}  // namespace

enkf_status launch_localize(enkf_dtype dt, const LocalizeArgs& a, hipStream_t s) {
  if (a.n_state <= 0 || a.N <= 0) return ENKF_SUCCESS;
  if (a.N <= L6_K) {
    const int64_t rb = (a.n_state + L6_TI - 1) / L6_TI;
    if (rb > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "localized analysis: grid too large");
    if (dt == ENKF_F64) localize64_kernel<double><<<(unsigned)rb, LZ_NT, 0, s>>>(a);
    else localize64_kernel<float><<<(unsigned)rb, LZ_NT, 0, s>>>(a);
    ENKF_HIP_CHECK(hipGetLastError());
    return ENKF_SUCCESS;
  }
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
