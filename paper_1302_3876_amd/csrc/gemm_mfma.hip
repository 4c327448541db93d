// Matrix-core products of the blocked solve, the refinement residual and the
// analysis update, for gfx950.
//
//  tn: P = A^T B over the n observations, A: n x a, B: n x m, column-major,
//      split over row chunks; every chunk writes an a x m partial and a
//      second kernel sums the partials in chunk order (deterministic).
//      (the panel products V_K^T [U_K, X] of the Woodbury identity, eq. SWM,
//      and G = V^T Z of the analysis and of the residual)
//  nn: tall products with a short inner dimension K:
//      UPDATE    X   <- X - A Bm                   (X -= U_K Q, the panel update)
//      ANALYSIS  XA  <- XB + (XB - xbar 1^T)(s Bm) (X^A = X^B + S V^T Z, Section 3.1)
//      RESIDUAL  RHO <- D - (r o Z + A Bm)         (D - W Z with Bm = V^T Z)
//      Bm is FP64 (it comes from the FP64 panel factorisation or from the
//      FP64 products) and is rounded to the MFMA input type when staged.
//
// tn: 2 x WA waves (FP64 8, FP32 4), block tile 128 (m) x 32 WA (a), wave
// tile 64 x 32. nn: 4 waves (2 x 2), tiles of 64 x 128 when the product has
// at most 128 columns, else 128 x 64 (FP64) or 128 x 128 (FP32). Both stage
// the inner dimension in steps of KC through one LDS buffer, the next step
// loaded into registers (16-byte global loads) while the matrix cores work on
// the current one. tn stages both operands k-contiguous ([col][k], 16-byte
// rows); nn stages A row-contiguous ([k][row]) so its global reads and LDS
// writes are both along rows. MFMA result lanes run along the output's
// leading dimension, so stores are coalesced.
//  analysis_small: the ANALYSIS product for N <= 96 (FP64) / 128 (FP32):
//      persistent 8-wave blocks with the whole right factor in the LDS, each
//      X^B row tile read once (left factor, row means and epilogue input).
#include <atomic>

#include "enkf_internal.h"
#include "gemm_mfma.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int NT = 256;  // 4 waves
constexpr int TILE = 128;

template <typename T> struct MfOf;
template <> struct MfOf<double> { typedef MfmaF64 type; };
template <> struct MfOf<float> { typedef MfmaF32 type; };

// 16-byte vectors
template <typename T> struct V16;
template <> struct V16<double> { static constexpr int W = 2; typedef double type __attribute__((ext_vector_type(2))); };
template <> struct V16<float> { static constexpr int W = 4; typedef float type __attribute__((ext_vector_type(4))); };

template <typename T> constexpr int kc_of() { return sizeof(T) == 8 ? 16 : 32; }

// Staged global loads are branch-free: an index outside the valid range is
// replaced by a valid one, and where the value matters the staged value is
// replaced by zero when it is written to LDS (after the matrix-core work of
// the current stage, so the loads stay in flight meanwhile). Branches around
// loads, or selects right after them, make the compiler wait for every load
// in flight and serialise the prefetch.
// VEC: 16-byte loads; the launcher guarantees 16-byte aligned columns and a
// row limit that is a multiple of W, so a vector is wholly inside or wholly
// outside the valid rows.
template <typename T, bool VEC>
__device__ __forceinline__ typename V16<T>::type load_rows(const T* __restrict__ col, int64_t row, int64_t rlim) {
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  vt v;
  if constexpr (VEC) {
    v = *reinterpret_cast<const vt*>(col + (row < rlim ? row : 0));
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = col[row + e < rlim ? row + e : 0];
  }
  return v;
}

// Zero the elements of v at rows >= rlim.
template <typename T>
__device__ __forceinline__ typename V16<T>::type zero_past(typename V16<T>::type v, int64_t row, int64_t rlim) {
  constexpr int W = V16<T>::W;
#pragma unroll
  for (int e = 0; e < W; ++e) v[e] = row + e < rlim ? v[e] : T(0);
  return v;
}

// ---------------------------------------------------------------- tn
// Stage layout: S[col][k], col in [0, TA + TILE) (A columns then B columns),
// k in [0, KC), row stride LDK (KC+4 / KC+2: 16-byte rows). One LDS buffer:
// the next stage is prefetched into registers while the matrix cores work on
// the current one. The inner dimension is taken in groups of 4 RV rows (RV =
// 2): lane group g = l/16 supplies rows RV g .. RV g + RV-1 of the group to
// RV consecutive MFMAs, read with one LDS load (the sum over the group is the
// same in any order of its rows).
template <typename T> constexpr int tn_ldk() { return sizeof(T) == 8 ? kc_of<T>() + 2 : kc_of<T>() + 4; }

// 2 x WA waves, wave tile 64 (m) x 32 (a) = 4 x 2 MFMA tiles; block tile
// 128 (m) x TA = 32*WA (a). FP64: WA = 4 (two 8-wave blocks per CU); FP32:
// WA = 2 (its FP64 flush accumulators need more registers: three 4-wave
// blocks per CU).
template <typename T> constexpr int tn_wa() { return sizeof(T) == 8 ? 4 : 2; }

template <typename T, bool VEC, int WA>
__global__ __launch_bounds__(128 * WA, WA == 2 ? 3 : 4) void tn_partial_kernel(int64_t n, int a, int m, const T* __restrict__ A, int64_t lda,
                                                        const T* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ partial, int64_t rows_per_chunk,
                                                        int tiles_m) {
  typedef typename MfOf<T>::type MF;
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  constexpr int KC = kc_of<T>();
  constexpr int LDK = tn_ldk<T>();
  constexpr int RV = 2;                           // inner-dimension rows per operand read
  typedef T rvt __attribute__((ext_vector_type(RV)));
  constexpr int TN_NT = 128 * WA;
  constexpr int TA = 32 * WA;
  constexpr int COLS = TA + TILE;
  constexpr int PER_COL = KC / W;                 // 16-byte loads per column per stage
  constexpr int COLS_PER_PASS = TN_NT / PER_COL;
  constexpr int PASSES = COLS / COLS_PER_PASS;
  __shared__ T S[COLS * LDK];

  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * TA, m0 = tm * TILE;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int m_off = (w / WA) * 64, a_off = (w % WA) * 32;
  const int lc = t / PER_COL, lk = (t % PER_COL) * W;

  // this thread's staged columns; a column outside the operand is replaced by
  // its last column (it only feeds outputs that are not stored)
  const T* cp[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const int c = p * COLS_PER_PASS + lc;
    if (c < TA) cp[p] = A + (int64_t)min(a0 + c, a - 1) * lda;
    else cp[p] = B + (int64_t)min(m0 + c - TA, m - 1) * ldb;
  }

  typename MF::acc_t acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();
  // FP32 accumulators are emptied into FP64 ones every kFlush stages, so no
  // FP32 sum runs over more than kFlush*KC rows (long FP32 sums over the
  // observations would otherwise dominate the error of the mixed solve).
  constexpr bool kWide = sizeof(T) == 4;
  constexpr int kFlush = 2;
  double wide[kWide ? 4 : 1][kWide ? 2 : 1][kWide ? 4 : 1] = {};
  auto flush = [&]() {
    if constexpr (kWide) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) wide[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = MF::zero();
        }
    }
  };

  vt reg[PASSES];
  // fetch is unconditional (past the chunk it reads row 0 again, discarded)
  auto fetch = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) reg[p] = load_rows<T, VEC>(cp[p], rs + lk, r1);
  };
  auto stash = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      T* dst = &S[(p * COLS_PER_PASS + lc) * LDK + lk];
      const vt v = zero_past<T>(reg[p], rs + lk, r1);
      if constexpr (LDK % W == 0) {
        *reinterpret_cast<vt*>(dst) = v;
      } else {
#pragma unroll
        for (int e = 0; e < W; ++e) dst[e] = v[e];
      }
    }
  };

  if (r0 < r1) {
    fetch(r0);
    stash(r0);
  }
  __syncthreads();
  int stage = 0;
  for (int64_t rs = r0; rs < r1; rs += KC) {
    fetch(rs + KC);
    // keep the prefetch ahead of the matrix-core work (the scheduler would
    // otherwise sink the loads next to their first use)
    __builtin_amdgcn_sched_barrier(0);
    const T* Sa = &S[0];
    const T* Sb = &S[TA * LDK];
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4 * RV) {
      rvt bq[4], aq[2];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        bq[i] = *reinterpret_cast<const rvt*>(&Sb[(m_off + 16 * i + l % 16) * LDK + kk + RV * (l / 16)]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        aq[j] = *reinterpret_cast<const rvt*>(&Sa[(a_off + 16 * j + l % 16) * LDK + kk + RV * (l / 16)]);
#pragma unroll
      for (int e = 0; e < RV; ++e)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = MF::mma(bq[i][e], aq[j][e], acc[i][j]);
    }
    if (kWide && ++stage == kFlush) {
      flush();
      stage = 0;
    }
    // unconditional (after the last stage it stages zeros): a conditional
    // stash would let the compiler sink the prefetch into the condition; the
    // scheduling barrier keeps the stash's use of the loads after the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(rs + KC);
    __syncthreads();
  }
  flush();
  // acc[i][j] element (row = m index, col = a index)
  double* P = partial + (int64_t)blockIdx.x * a * m;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mi = m0 + m_off + 16 * i + MF::row(l, r);
        const int ai = a0 + a_off + 16 * j + l % 16;
        if (mi < m && ai < a) P[ai + (int64_t)mi * a] = kWide ? wide[i][j][r] : (double)acc[i][j][r];
      }
}

// Sum of the chunk partials: block = 64 outputs x 4 waves; wave w sums the
// chunks w, w+4, ... in order, then the four wave sums are added in order.
__global__ __launch_bounds__(256) void partial_sum_kernel(int a, int m, int64_t chunks, const double* __restrict__ partial,
                                                          double* __restrict__ G, int64_t ldg) {
  __shared__ double red[4][64];
  const int64_t am = (int64_t)a * m;
  const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x % 64;
  const int w = threadIdx.x / 64;
  // wave w sums the chunks w, w + 4, ... into 8 running sums (chunk
  // w + 4 (8 q + u) goes to sum u), added in order at the end
  constexpr int U = 8;
  double su[U] = {};
  const int64_t ec = e < am ? e : am - 1;
  int64_t c = w;
  for (; c + 4 * (U - 1) < chunks; c += 4 * U) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = partial[(c + 4 * u) * am + ec];
#pragma unroll
    for (int u = 0; u < U; ++u) su[u] += x[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (c + 4 * u < chunks) su[u] += partial[(c + 4 * u) * am + ec];
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) s += su[u];
  red[w][threadIdx.x % 64] = s;
  __syncthreads();
  if (w == 0 && e < am) {
    const int q = threadIdx.x;
    const double tot = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    const int i = (int)(e % a), j = (int)(e / a);
    G[i + (int64_t)j * ldg] = tot;
  }
}

// ---------------------------------------------------------------- nn
// The right factor, scale * Bm, is converted once per call to the storage
// type and laid out row-major, Bt[k * ldbc + j], with zero padding to
// nn_bt_rows(K) rows and nn_bt_cols(m) columns: every stage of every tile
// reads it without bounds checks, 16 bytes at a time.
template <typename T>
__global__ __launch_bounds__(256) void convert_b_kernel(int K, int m, const double* __restrict__ Bm, int64_t ldb,
                                                        double scale, T* __restrict__ Bt, int rows, int ldbc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * ldbc) return;
  const int j = (int)(e % ldbc), k = (int)(e / ldbc);
  Bt[e] = (k < K && j < m) ? (T)(scale * Bm[k + (int64_t)j * ldb]) : T(0);
}

// Stage layout: As[k][row] (row stride TR+16), Bs[k][col] (stride TC+16):
// 16-byte LDS writes along rows/columns, conflict-free MFMA operand reads.
// Waves 2 x 2: wave (w/2, w%2) owns TC/2 columns x TR/2 rows. One LDS
// buffer; the next stage is prefetched into registers.
// A budget of two waves per SIMD lets the compiler keep the accumulators in
// VGPRs; with the default one it split them from the MFMA operands into the
// accumulation registers (FP64: copied in and out around every stage's
// MFMAs) and needed more registers in all, so fewer waves fit.
template <typename T, int MODE, int TR, int TC, bool VEC, bool LOOP>
__global__ __launch_bounds__(NT, 2) void nn_kernel(NnArgs p, const T* __restrict__ Bt, int ldbc) {
  static_assert(!LOOP || MODE == NN_ANALYSIS, "only ANALYSIS walks the column tiles");
  typedef typename MfOf<T>::type MF;
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  constexpr int KC = kc_of<T>();
  constexpr int CI = TC / 32;                     // MFMA column tiles per wave
  constexpr int RJ = TR / 32;                     // MFMA row tiles per wave
  constexpr int LDR = TR + 16;
  constexpr int LDC = TC + 16;
  constexpr int ROWCH = TR / W;                   // 16-byte loads per k of the A tile
  constexpr int A_PASSES = (KC * ROWCH) / NT;
  constexpr int COLCH = TC / W;                   // 16-byte loads per k of the B stage
  constexpr int B_PASSES = (KC * COLCH) / NT;
  static_assert(A_PASSES >= 1 && B_PASSES >= 1, "tile too small for the block");
  __shared__ T As[KC * LDR];
  __shared__ T Bs[KC * LDC];
  __shared__ double mean[TR];
  int64_t rt;
  int ct;
  // LOOP: one block takes every column tile of its row tile (the row means of
  // ANALYSIS are then formed once per row tile). It is a separate instance so
  // that one-tile launches keep their register budget (occupancy).
  xcd_tile_map(blockIdx.x, p.n_row_tiles, LOOP ? 1 : p.n_col_tiles, &rt, &ct);
  if (rt >= p.n_row_tiles) {
    // a padding block of the grid: its share of ||rho||^2 is zero
    if (MODE == NN_RESIDUAL && p.part && threadIdx.x == 0) p.part[blockIdx.x] = 0.0;
    return;
  }
  const int64_t row0 = rt * TR;
  const T* __restrict__ A = static_cast<const T*>(p.A);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int c_off = (w / 2) * (TC / 2), r_off = (w % 2) * (TR / 2);
  const int64_t rlim = p.n;
  const int bt_rows = (p.K + 31) / 32 * 32;   // rows of Bt (nn_bt_rows)

  if constexpr (MODE == NN_ANALYSIS) {
    // row means of the block's rows: NT/TR partial sums per row, each over a
    // fixed subset of the columns, added in a fixed order
    constexpr int Q = NT / TR;
    constexpr int U = 8;
    __shared__ double part[Q][TR];
    const int rr = t % TR, q = t / TR;
    const int64_t row = min(row0 + rr, rlim - 1);
    const T* __restrict__ ar = A + row;
    double s = 0.0;
    int j = q;
    for (; j + (U - 1) * Q < p.K; j += U * Q) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = ar[(int64_t)(j + u * Q) * p.lda];
#pragma unroll
      for (int u = 0; u < U; ++u) s += (double)x[u];
    }
    for (; j < p.K; j += Q) s += (double)ar[(int64_t)j * p.lda];
    part[q][rr] = s;
    __syncthreads();
    if (t < TR) {
      double tot = 0.0;
#pragma unroll
      for (int z = 0; z < Q; ++z) tot += part[z][t];
      mean[t] = tot / (double)p.K;
    }
    __syncthreads();
  }

  const int ct_end = LOOP ? p.n_col_tiles : ct + 1;
  for (; ct < ct_end; ++ct) {
  const int col0 = ct * TC;
  typename MF::acc_t acc[CI][RJ];
#pragma unroll
  for (int i = 0; i < CI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) acc[i][j] = MF::zero();

  vt areg[A_PASSES];
  vt breg[B_PASSES];
  // fetch is unconditional: a column index past K reads column K-1 (zeroed
  // when staged; Bt is zero there as well); rows past n only feed outputs
  // that are not stored
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / ROWCH, rc = (e % ROWCH) * W;
      const int k = min(k0 + kk, p.K - 1);
      areg[q] = load_rows<T, VEC>(A + (int64_t)k * p.lda, row0 + rc, rlim);
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / COLCH, cc = (e % COLCH) * W;
      const int k = min(k0 + kk, bt_rows - 1);
      breg[q] = *reinterpret_cast<const vt*>(Bt + (int64_t)k * ldbc + col0 + cc);
    }
  };
  auto stash = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / ROWCH, rc = (e % ROWCH) * W;
      const bool kok = k0 + kk < p.K;
      vt v = areg[q];
#pragma unroll
      for (int x = 0; x < W; ++x) {
        if constexpr (MODE == NN_ANALYSIS) v[x] = (T)((double)v[x] - mean[rc + x]);
        v[x] = kok ? v[x] : T(0);
      }
      *reinterpret_cast<vt*>(&As[kk * LDR + rc]) = v;
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / COLCH, cc = (e % COLCH) * W;
      *reinterpret_cast<vt*>(&Bs[kk * LDC + cc]) = breg[q];
    }
  };

  fetch(0);
  stash(0);
  __syncthreads();
  for (int k0 = 0; k0 < p.K; k0 += KC) {
    fetch(k0 + KC);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < KC; kk += MF::KSTEP) {
      T cop[CI], rop[RJ];
#pragma unroll
      for (int i = 0; i < CI; ++i) cop[i] = Bs[(kk + l / 16) * LDC + c_off + 16 * i + l % 16];
#pragma unroll
      for (int j = 0; j < RJ; ++j) rop[j] = As[(kk + l / 16) * LDR + r_off + 16 * j + l % 16];
#pragma unroll
      for (int i = 0; i < CI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = MF::mma(cop[i], rop[j], acc[i][j]);
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(k0 + KC);
    __syncthreads();
  }
  // acc[i][j] element (row = output column, col = output row). The inputs of
  // the epilogue are loaded for all of the wave's outputs first (clamped
  // indices, no branches), so their latencies overlap; stores are predicated.
  const T* __restrict__ Cin = static_cast<const T*>(p.Cin);
  const T* __restrict__ Din = static_cast<const T*>(p.Din);
  T* __restrict__ Cout = static_cast<T*>(p.Cout);
  double ss = 0.0;   // RESIDUAL: this thread's sum of the stored rho^2
  // RESIDUAL loads two inputs per output: its rows go in two halves, so the
  // prefetched inputs leave registers for a third wave per SIMD
  constexpr int JG = (MODE == NN_RESIDUAL || MODE == NN_UPDATE64) && RJ % 2 == 0 ? RJ / 2 : RJ;
#pragma unroll
  for (int i = 0; i < CI; ++i) {
#pragma unroll
  for (int jg = 0; jg < RJ; jg += JG) {
    T cin[JG][4], din[JG][4];
    double rr[JG], zin[JG][4];
#pragma unroll
    for (int jj = 0; jj < JG; ++jj) {
      const int j = jg + jj;
      const int64_t row = min(row0 + r_off + 16 * j + l % 16, rlim - 1);
      if constexpr (MODE == NN_RESIDUAL) rr[jj] = p.r[row];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = min(col0 + c_off + 16 * i + MF::row(l, r), p.m - 1);
        cin[jj][r] = Cin[row + (int64_t)col * p.ldc];
        if constexpr (MODE == NN_RESIDUAL) din[jj][r] = Din[row + (int64_t)col * p.ldd];
        if constexpr (MODE == NN_UPDATE64) zin[jj][r] = p.z64_acc ? p.Z64[row + (int64_t)col * p.ldz64] : 0.0;
      }
    }
#pragma unroll
    for (int jj = 0; jj < JG; ++jj) {
      const int j = jg + jj;
      double rinv = 1.0;
      if constexpr (MODE == NN_RESIDUAL) rinv = 1.0 / rr[jj];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + c_off + 16 * i + MF::row(l, r);
        const int64_t row = row0 + r_off + 16 * j + l % 16;
        const double prod = (double)acc[i][j][r];
        const double c = (double)cin[jj][r];
        double out;
        if constexpr (MODE == NN_UPDATE || MODE == NN_UPDATE64) out = c - prod;
        else if constexpr (MODE == NN_ANALYSIS) out = c + prod;
        else out = (double)din[jj][r] - (rr[jj] * c + prod);
        const bool in = col < p.m && row < p.n;
        if constexpr (MODE == NN_RESIDUAL) {
          // the right-hand side of the next low-precision solve, Step 1
          // applied, or rho itself
          if (in) {
            if (p.Cout32) p.Cout32[row + (int64_t)col * p.ldo32] = (float)(out * rinv);
            else Cout[row + (int64_t)col * p.ldo] = (T)out;
          }
          ss += in ? out * out : 0.0;
        } else if constexpr (MODE == NN_UPDATE64) {
          if (in) p.Z64[row + (int64_t)col * p.ldz64] = zin[jj][r] + out;
        } else {
          if (in) Cout[row + (int64_t)col * p.ldo] = (T)out;
        }
      }
    }
  }
  }
  if constexpr (MODE == NN_RESIDUAL) {
    // the block's share of ||rho||^2: lanes, then the 4 waves, in a fixed order
    if (p.part) {
      static_assert(NT == 4 * kWave, "four waves per block");
      __shared__ double red[4];
      for (int off = kWave / 2; off > 0; off >>= 1) ss += __shfl_xor(ss, off, kWave);
      if (l == 0) red[w] = ss;
      __syncthreads();
      if (t == 0) p.part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
  }
  }
}

// out[0] = sum of part[0..count) in a fixed order (one block).
__global__ __launch_bounds__(256) void part_sum_kernel(int64_t count, const double* __restrict__ part,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < count; b += 256) s += part[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------- analysis, small N
// X^A = X^B + (X^B - xbar 1^T) B for N = K = m <= 16 NT16 (NT16 even, so
// NP = 16 NT16 = nn_bt_rows(N)). Persistent blocks walk row tiles of 64
// rows; the block keeps all of B (NP x NP, from Bt) in the LDS and reads
// each X^B row tile from HBM once: the tile is staged in the LDS (it is the
// left factor, its row means and the epilogue's X^B); the block's next two
// tiles are in flight in registers while the matrix cores work.
// 8 waves: wave w forms the output rows 16 (w % 4) .. for half of the
// column tiles.
constexpr int AS_TR = 64;

constexpr int AS_NT = 512;                        // 8 waves: two per SIMD

template <typename T, int NT16>
__global__ __launch_bounds__(AS_NT) void analysis_small_kernel(NnArgs p, const T* __restrict__ Bt, int ldbc) {
  typedef typename MfOf<T>::type MF;
  constexpr int NP = 16 * NT16;
  constexpr int LDB = NP + 4;                     // Bs[k][col]
  constexpr int LDX = AS_TR + 4;                  // Xs[col][row]
  constexpr int QS = AS_NT / AS_TR;               // threads per row when staging (8)
  constexpr int PX = NP / QS;                     // staged tile elements per thread
  constexpr int HC = NT16 / 2;                    // column tiles per wave
  __shared__ T Bs[NP * LDB];
  __shared__ T Xs[NP * LDX];
  __shared__ double part[QS][AS_TR];
  const T* __restrict__ X = static_cast<const T*>(p.A);
  T* __restrict__ XA = static_cast<T*>(p.Cout);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int N = p.K;
  const int64_t n = p.n;
  const int64_t tiles = (n + AS_TR - 1) / AS_TR;
  for (int e = t; e < NP * NP; e += AS_NT) {       // B: rows and columns past N are zero in Bt
    const int k = e / NP, c = e % NP;
    Bs[k * LDB + c] = Bt[(int64_t)k * ldbc + c];
  }
  // staged element q of this thread: row t % 64, column t / 64 + 8 q
  const int xr = t % AS_TR, xc = t / AS_TR;
  // wave w: output rows 16 (w % 4) .., column tiles (w / 4) HC ..
  const int ro = 16 * (w % 4) + l % 16;
  const int ct0 = (w / 4) * HC;
  auto fetch = [&](T (&xreg)[PX], int64_t tile) {
    const int64_t row = min(tile * AS_TR + xr, n - 1);
#pragma unroll
    for (int q = 0; q < PX; ++q) xreg[q] = X[row + (int64_t)min(xc + QS * q, N - 1) * p.lda];
  };
  // one row tile from the registers xreg, which then load the tile two
  // steps ahead
  auto process = [&](T (&xreg)[PX], int64_t tile) {
    __syncthreads();                               // the previous tile's epilogue is done with Xs
    {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < PX; ++q) {
        const int c = xc + QS * q;
        const T v = c < N ? xreg[q] : T(0);
        Xs[c * LDX + xr] = v;
        s += (double)v;
      }
      part[xc][xr] = s;
    }
    __syncthreads();
    if (tile + 2 * (int64_t)gridDim.x < tiles) fetch(xreg, tile + 2 * (int64_t)gridDim.x);
    __builtin_amdgcn_sched_barrier(0);
    double msum = 0.0;
#pragma unroll
    for (int z = 0; z < QS; ++z) msum += part[z][ro];
    const double mean = msum / (double)N;
    typename MF::acc_t acc[HC];
#pragma unroll
    for (int i = 0; i < HC; ++i) acc[i] = MF::zero();
    // rows k >= N of Bs are zero, so the left factor needs no mask there
#pragma unroll 8
    for (int k = 0; k < NP; k += MF::KSTEP) {
      const int kk = k + l / 16;
      const T aop = (T)((double)Xs[kk * LDX + ro] - mean);
#pragma unroll
      for (int i = 0; i < HC; ++i) acc[i] = MF::mma(Bs[kk * LDB + 16 * (ct0 + i) + l % 16], aop, acc[i]);
    }
    const int64_t row = tile * AS_TR + ro;
#pragma unroll
    for (int i = 0; i < HC; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * (ct0 + i) + MF::row(l, r);
        const double out = (double)Xs[min(col, NP - 1) * LDX + ro] + (double)acc[i][r];
        if (col < N && row < n) XA[row + (int64_t)col * p.ldo] = (T)out;
      }
  };
  T xa[PX], xb[PX];
  const int64_t G = gridDim.x;
  if ((int64_t)blockIdx.x < tiles) fetch(xa, blockIdx.x);
  if ((int64_t)blockIdx.x + G < tiles) fetch(xb, blockIdx.x + G);
  for (int64_t tile = blockIdx.x; tile < tiles; tile += 2 * G) {
    process(xa, tile);
    if (tile + G < tiles) process(xb, tile + G);
  }
}

template <typename T, int NT16>
enkf_status analysis_small_go(NnArgs p, const T* Bt, int ldbc, hipStream_t s) {
  // resident blocks per CU and the CU count, found on the first call (any
  // thread may find them; they are the same for every device of the part)
  static std::atomic<int> occ_a{0}, cus_a{0};
  int occ = occ_a.load(std::memory_order_relaxed), cus = cus_a.load(std::memory_order_relaxed);
  if (occ == 0 || cus == 0) {
    int b = 0, dev = 0, c = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, analysis_small_kernel<T, NT16>, AS_NT, 0) != hipSuccess ||
        b < 1)
      b = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = 256;
    occ = b;
    cus = c;
    occ_a.store(b, std::memory_order_relaxed);
    cus_a.store(c, std::memory_order_relaxed);
  }
  const int64_t tiles = (p.n + AS_TR - 1) / AS_TR;
  const int64_t blocks = std::min<int64_t>(tiles, (int64_t)cus * occ);
  analysis_small_kernel<T, NT16><<<(unsigned)blocks, AS_NT, 0, s>>>(p, Bt, ldbc);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

// N (= K = m) for which the small-N analysis kernel applies: its LDS holds
// B and one row tile.
template <typename T>
bool analysis_small_fits(int N) {
  return N >= 2 && N <= (sizeof(T) == 8 ? 96 : 128);
}

template <typename T>
enkf_status analysis_small(NnArgs p, const T* Bt, int ldbc, hipStream_t s) {
  const int nt16 = 2 * ((p.K + 31) / 32);
  switch (nt16) {
    case 2: return analysis_small_go<T, 2>(p, Bt, ldbc, s);
    case 4: return analysis_small_go<T, 4>(p, Bt, ldbc, s);
    case 6: return analysis_small_go<T, 6>(p, Bt, ldbc, s);
    default:
      if constexpr (sizeof(T) == 4) return analysis_small_go<T, 8>(p, Bt, ldbc, s);
      return fail(ENKF_ERR_NOT_SUPPORTED, "analysis: ensemble too large for the small-N kernel");
  }
}

constexpr int64_t kTnTargetBlocks = 768;   // ~3 blocks per CU
constexpr int64_t kTnMinRows = 64;

// Row chunks of a split-K product: enough blocks to fill the part, at least
// kTnMinRows rows each, and no more partials (chunks x a x m, FP64) than
// about twice the operands' elements (n x (a + m)), so that for short,
// wide products the partial sums do not outweigh the product.
int64_t tn_chunks(int64_t n, int a, int m) {
  const int64_t tiles = (int64_t)((a + TILE - 1) / TILE) * ((m + TILE - 1) / TILE);
  int64_t chunks = (kTnTargetBlocks + tiles - 1) / tiles;
  const int64_t max_rows = (n + kTnMinRows - 1) / kTnMinRows;
  const int64_t max_partials = std::max<int64_t>(4, 2 * n * ((int64_t)a + m) / ((int64_t)a * m));
  const int64_t max_chunks = std::min(max_rows, max_partials);
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  return chunks;
}

bool aligned16(const void* p, int64_t ld, size_t es) {
  return ((uintptr_t)p % 16) == 0 && ((ld * (int64_t)es) % 16) == 0;
}

}  // namespace

int64_t tn_partial_elems(int64_t n, int a, int m) { return tn_chunks(n, a, m) * (int64_t)a * m; }

enkf_status launch_tn(enkf_dtype dt, int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb,
                      double* G, int64_t ldg, double* partial, hipStream_t s) {
  if (a <= 0 || m <= 0) return ENKF_SUCCESS;
  const int64_t chunks = tn_chunks(n, a, m);
  const int kc = dt == ENKF_F64 ? kc_of<double>() : kc_of<float>();
  int64_t rpc = (n + chunks - 1) / chunks;
  rpc = ((rpc + kc - 1) / kc) * kc;
  const int64_t used = (n + rpc - 1) / rpc;
  const int tiles_m = (m + TILE - 1) / TILE;
  const size_t es = dt == ENKF_F64 ? 8 : 4;
  const int W = 16 / (int)es;
  const bool vec = aligned16(A, lda, es) && aligned16(B, ldb, es) && n % W == 0;
  if (dt == ENKF_F64) {
    constexpr int WA = tn_wa<double>();
    const int tiles = ((a + 32 * WA - 1) / (32 * WA)) * tiles_m;
    if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
    dim3 grid((unsigned)used, (unsigned)tiles);
    const double* a_ = static_cast<const double*>(A);
    const double* b_ = static_cast<const double*>(B);
    if (vec) tn_partial_kernel<double, true, WA><<<grid, 128 * WA, 0, s>>>(n, a, m, a_, lda, b_, ldb, partial, rpc, tiles_m);
    else tn_partial_kernel<double, false, WA><<<grid, 128 * WA, 0, s>>>(n, a, m, a_, lda, b_, ldb, partial, rpc, tiles_m);
  } else {
    constexpr int WA = tn_wa<float>();
    const int tiles = ((a + 32 * WA - 1) / (32 * WA)) * tiles_m;
    if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
    dim3 grid((unsigned)used, (unsigned)tiles);
    const float* a_ = static_cast<const float*>(A);
    const float* b_ = static_cast<const float*>(B);
    if (vec) tn_partial_kernel<float, true, WA><<<grid, 128 * WA, 0, s>>>(n, a, m, a_, lda, b_, ldb, partial, rpc, tiles_m);
    else tn_partial_kernel<float, false, WA><<<grid, 128 * WA, 0, s>>>(n, a, m, a_, lda, b_, ldb, partial, rpc, tiles_m);
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return launch_partial_sum(a, m, used, partial, G, ldg, s);
}

enkf_status launch_partial_sum(int a, int m, int64_t chunks, const double* partial, double* G, int64_t ldg,
                               hipStream_t s) {
  const int64_t am = (int64_t)a * m;
  partial_sum_kernel<<<(unsigned)((am + 63) / 64), 256, 0, s>>>(a, m, chunks, partial, G, ldg);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

constexpr int64_t kNnLoopRowTiles = 2048;   // ~8 row tiles per CU

// rows: a multiple of the largest stage depth (32); columns: of the widest tile (128)
int nn_bt_rows(int K) { return (K + 31) / 32 * 32; }
int nn_bt_cols(int m) { return (m + 127) / 128 * 128; }

// the largest RESIDUAL grid: row tiles of 64 (m <= 128) or 128, padded to a
// multiple of 8, times column tiles of at least 64
int64_t nn_residual_part_elems(int64_t n, int m) {
  return ((n + 63) / 64 + 7) / 8 * 8 * std::max<int64_t>(1, ((int64_t)m + 63) / 64);
}

size_t nn_bt_bytes(int K, int m) { return sizeof(double) * (size_t)nn_bt_rows(K) * (size_t)nn_bt_cols(m); }

namespace {

template <typename T, int MODE, int TR, int TC>
enkf_status nn_go(NnArgs p, const T* Bt, int ldbc, bool vec, hipStream_t s) {
  p.n_row_tiles = (p.n + TR - 1) / TR;
  p.n_col_tiles = (p.m + TC - 1) / TC;
  // ANALYSIS with several column tiles and rows enough to fill the part: one
  // block per row tile walks its column tiles (row means formed once)
  const bool loop = MODE == NN_ANALYSIS && p.n_col_tiles > 1 && p.n_row_tiles >= kNnLoopRowTiles;
  const int64_t groups = (p.n_row_tiles + 7) / 8;
  const int64_t blocks = groups * 8 * (loop ? 1 : p.n_col_tiles);
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "nn product: grid too large");
  if constexpr (MODE == NN_RESIDUAL) {
    if (p.part && (blocks > p.part_cap || !p.sumsq))
      return fail(ENKF_ERR_INVALID_ARG, "residual product: norm partials too small or no output");
  }
  if constexpr (MODE == NN_ANALYSIS && TR == 128) {   // the tiles taken when m > 128
    if (loop) {
      if (vec) nn_kernel<T, MODE, TR, TC, true, true><<<(unsigned)blocks, NT, 0, s>>>(p, Bt, ldbc);
      else nn_kernel<T, MODE, TR, TC, false, true><<<(unsigned)blocks, NT, 0, s>>>(p, Bt, ldbc);
      ENKF_HIP_CHECK(hipGetLastError());
      return ENKF_SUCCESS;
    }
  }
  if (vec) nn_kernel<T, MODE, TR, TC, true, false><<<(unsigned)blocks, NT, 0, s>>>(p, Bt, ldbc);
  else nn_kernel<T, MODE, TR, TC, false, false><<<(unsigned)blocks, NT, 0, s>>>(p, Bt, ldbc);
  ENKF_HIP_CHECK(hipGetLastError());
  if constexpr (MODE == NN_RESIDUAL) {
    if (p.part) {
      part_sum_kernel<<<1, 256, 0, s>>>(blocks, p.part, p.sumsq);
      ENKF_HIP_CHECK(hipGetLastError());
    }
  }
  return ENKF_SUCCESS;
}

// Tile choice: one column tile of 128 when m <= 128 (64 rows), else
// 128 rows x 64 (FP64) or 128 (FP32) columns.
template <typename T, int MODE>
enkf_status nn_pick(NnArgs p, const T* Bt, int ldbc, bool vec, hipStream_t s) {
  if (p.m <= 128) return nn_go<T, MODE, 64, 128>(p, Bt, ldbc, vec, s);
  if constexpr (sizeof(T) == 8) return nn_go<T, MODE, 128, 64>(p, Bt, ldbc, vec, s);
  else return nn_go<T, MODE, 128, 128>(p, Bt, ldbc, vec, s);
}

template <typename T>
enkf_status nn_typed(int mode, NnArgs p, hipStream_t s) {
  T* Bt = static_cast<T*>(p.bws);
  const int rows = nn_bt_rows(p.K), ldbc = nn_bt_cols(p.m);
  const int64_t total = (int64_t)rows * ldbc;
  convert_b_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(p.K, p.m, p.Bm, p.ldb, p.scale, Bt, rows, ldbc);
  ENKF_HIP_CHECK(hipGetLastError());
  const bool vec = aligned16(p.A, p.lda, sizeof(T)) && p.n % (int64_t)(16 / sizeof(T)) == 0;
  if (mode == NN_UPDATE) return nn_pick<T, NN_UPDATE>(p, Bt, ldbc, vec, s);
  if (mode == NN_UPDATE64) {
    if constexpr (sizeof(T) == 4) {
      if (!p.Z64) return fail(ENKF_ERR_INVALID_ARG, "update product: no FP64 destination");
      return nn_pick<T, NN_UPDATE64>(p, Bt, ldbc, vec, s);
    } else {
      return fail(ENKF_ERR_NOT_SUPPORTED, "update product into FP64: FP32 storage only");
    }
  }
  if (mode == NN_ANALYSIS) {
    if (p.K == p.m && p.Cin == p.A && p.ldc == p.lda && analysis_small_fits<T>(p.K))
      return analysis_small<T>(p, Bt, ldbc, s);
    return nn_pick<T, NN_ANALYSIS>(p, Bt, ldbc, vec, s);
  }
  // the refinement residual is formed in FP64 only
  if constexpr (sizeof(T) == 8) return nn_pick<T, NN_RESIDUAL>(p, Bt, ldbc, vec, s);
  else return fail(ENKF_ERR_NOT_SUPPORTED, "residual product: FP64 only");
}

}  // namespace

enkf_status launch_nn(enkf_dtype dt, int mode, NnArgs p, hipStream_t s) {
  if (p.n <= 0 || p.m <= 0) return ENKF_SUCCESS;
  if (!p.bws) return fail(ENKF_ERR_INVALID_ARG, "nn product: no workspace for the converted right factor");
  if (dt == ENKF_F64) return nn_typed<double>(mode, p, s);
  return nn_typed<float>(mode, p, s);
}

}  // namespace enkf
