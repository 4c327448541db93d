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
// Both kernels: 256 threads (4 waves, 2 x 2); tn uses 128 x 128 output tiles
// (each wave 64 x 64 = 4 x 4 MFMA tiles), nn 64 x 128 when the product has at
// most 128 columns, else 128 x 64 (FP64) or 128 x 128 (FP32); inner-dimension stages of KC staged in LDS
// through registers with 16-byte global loads, double-buffered so the next
// stage's loads are in flight while the matrix cores work on the current one.
// tn stages both operands k-contiguous ([col][k], padded: conflict-free MFMA
// reads); nn stages A row-contiguous ([k][row]) so its global reads and LDS
// writes are both along rows. MFMA result lanes run along the output's
// leading dimension, so stores are coalesced.
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

// Load W consecutive elements of a column starting at row `row` (rows < rlim
// only; others are zero). `vec` says the 16-byte path is aligned.
template <typename T>
__device__ __forceinline__ typename V16<T>::type load_col_vec(const T* __restrict__ p, int64_t row, int64_t rlim,
                                                              bool vec) {
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  vt v;
  if (vec && row + W <= rlim) {
    v = *reinterpret_cast<const vt*>(p + row);
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = (row + e < rlim) ? p[row + e] : T(0);
  }
  return v;
}

// ---------------------------------------------------------------- tn
// Stage layout: S[col][k], col in [0, 2*TILE) (A columns then B columns),
// k in [0, KC), row stride KC+1.
template <typename T>
__global__ __launch_bounds__(NT) void tn_partial_kernel(int64_t n, int a, int m, const T* __restrict__ A, int64_t lda,
                                                        const T* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ partial, int64_t rows_per_chunk,
                                                        int tiles_m, bool vec) {
  typedef typename MfOf<T>::type MF;
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  constexpr int KC = kc_of<T>();
  constexpr int LDK = KC + 1;
  constexpr int COLS = 2 * TILE;
  constexpr int PER_COL = KC / W;                 // 16-byte loads per column per stage
  constexpr int COLS_PER_PASS = NT / PER_COL;
  constexpr int PASSES = COLS / COLS_PER_PASS;
  __shared__ T S[2][COLS * LDK];

  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * TILE, m0 = tm * TILE;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int m_off = (w / 2) * 64, a_off = (w % 2) * 64;
  const int lc = t / PER_COL, lk = (t % PER_COL) * W;

  // column pointers of this thread's staged columns (nullptr: outside)
  const T* cp[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const int c = p * COLS_PER_PASS + lc;
    if (c < TILE) cp[p] = (a0 + c < a) ? A + (int64_t)(a0 + c) * lda : nullptr;
    else cp[p] = (m0 + c - TILE < m) ? B + (int64_t)(m0 + c - TILE) * ldb : nullptr;
  }

  typename MF::acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = MF::zero();
  // FP32 accumulators are emptied into FP64 ones every kFlush stages, so no
  // FP32 sum runs over more than kFlush*KC rows (long FP32 sums over the
  // observations would otherwise dominate the error of the mixed solve).
  constexpr bool kWide = sizeof(T) == 4;
  constexpr int kFlush = 2;
  double wide[kWide ? 4 : 1][kWide ? 4 : 1][kWide ? 4 : 1] = {};
  auto flush = [&]() {
    if constexpr (kWide) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) wide[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = MF::zero();
        }
    }
  };

  vt reg[PASSES];
  auto fetch = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      if (cp[p]) reg[p] = load_col_vec<T>(cp[p], rs + lk, r1, vec);
      else {
#pragma unroll
        for (int e = 0; e < W; ++e) reg[p][e] = T(0);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      T* dst = &S[buf][(p * COLS_PER_PASS + lc) * LDK + lk];
#pragma unroll
      for (int e = 0; e < W; ++e) dst[e] = reg[p][e];
    }
  };

  int buf = 0;
  if (r0 < r1) {
    fetch(r0);
    stash(0);
  }
  __syncthreads();
  int stage = 0;
  for (int64_t rs = r0; rs < r1; rs += KC) {
    const bool more = rs + KC < r1;
    if (more) fetch(rs + KC);
    const T* Sa = &S[buf][0];
    const T* Sb = &S[buf][TILE * LDK];
#pragma unroll
    for (int kk = 0; kk < KC; kk += MF::KSTEP) {
      T bop[4], aop[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) bop[i] = Sb[(m_off + 16 * i + l % 16) * LDK + kk + l / 16];
#pragma unroll
      for (int j = 0; j < 4; ++j) aop[j] = Sa[(a_off + 16 * j + l % 16) * LDK + kk + l / 16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(bop[i], aop[j], acc[i][j]);
    }
    if (more) stash(buf ^ 1);
    if (kWide && ++stage == kFlush) {
      flush();
      stage = 0;
    }
    __syncthreads();
    buf ^= 1;
  }
  flush();
  // acc[i][j] element (row = m index, col = a index)
  double* P = partial + (int64_t)blockIdx.x * a * m;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
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
  double s = 0.0;
  if (e < am)
    for (int64_t c = w; c < chunks; c += 4) s += partial[c * am + e];
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
// B = scale * Bm converted once per call to the storage type, K padded to a
// multiple of 16 with zeros (so the kernel stages B without bounds checks on
// k and with 16-byte loads).
template <typename T>
__global__ __launch_bounds__(256) void convert_b_kernel(int K, int m, const double* __restrict__ Bm, int64_t ldb,
                                                        double scale, T* __restrict__ Bt, int ldbt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ldbt * m) return;
  const int k = (int)(e % ldbt), j = (int)(e / ldbt);
  Bt[e] = (k < K) ? (T)(scale * Bm[k + (int64_t)j * ldb]) : T(0);
}

// Stage layout: As[k][row] (row stride TR+1), Bs[k][col] (stride TC+1).
// Waves 2 x 2: wave (w/2, w%2) owns TC/2 columns x TR/2 rows.
template <typename T, int MODE, int TR, int TC>
__global__ __launch_bounds__(NT) void nn_kernel(NnArgs p, const T* __restrict__ Bt, int ldbt, bool vec) {
  typedef typename MfOf<T>::type MF;
  typedef typename V16<T>::type vt;
  constexpr int W = V16<T>::W;
  constexpr int KC = kc_of<T>();
  constexpr int CI = TC / 32;                     // MFMA column tiles per wave
  constexpr int RJ = TR / 32;                     // MFMA row tiles per wave
  constexpr int LDR = TR + 1;
  constexpr int LDC = TC + 1;
  constexpr int ROWCH = TR / W;                   // 16-byte loads per k column of the A tile
  constexpr int A_PASSES = (KC * ROWCH) / NT;
  constexpr int BCH = KC / W;                     // 16-byte loads per column of the B stage
  constexpr int B_PASSES = (TC * BCH) / NT;
  static_assert(A_PASSES >= 1 && B_PASSES >= 1, "tile too small for the block");
  __shared__ T As[2][KC * LDR];
  __shared__ T Bs[2][KC * LDC];
  __shared__ double mean[TR];
  int64_t rt;
  int ct;
  xcd_tile_map(blockIdx.x, p.n_row_tiles, p.n_col_tiles, &rt, &ct);
  if (rt >= p.n_row_tiles) return;
  const int64_t row0 = rt * TR;
  const int col0 = ct * TC;
  const T* __restrict__ A = static_cast<const T*>(p.A);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int c_off = (w / 2) * (TC / 2), r_off = (w % 2) * (TR / 2);
  const int64_t rlim = p.n;

  if constexpr (MODE == NN_ANALYSIS) {
    // row means of the block's rows (fixed order)
    constexpr int Q = NT / TR;
    __shared__ double part[Q][TR];
    const int rr = t % TR, q = t / TR;
    const int64_t row = row0 + rr;
    double s = 0.0;
    if (row < p.n)
      for (int j = q; j < p.K; j += Q) s += (double)A[row + (int64_t)j * p.lda];
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

  typename MF::acc_t acc[CI][RJ];
#pragma unroll
  for (int i = 0; i < CI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) acc[i][j] = MF::zero();

  vt areg[A_PASSES];
  vt breg[B_PASSES];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / ROWCH, rc = (e % ROWCH) * W;
      if (k0 + kk < p.K) {
        areg[q] = load_col_vec<T>(A + (int64_t)(k0 + kk) * p.lda, row0 + rc, rlim, vec);
      } else {
#pragma unroll
        for (int x = 0; x < W; ++x) areg[q][x] = T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int e = q * NT + t;
      const int cc = e / BCH, kk = (e % BCH) * W;
      if (col0 + cc < p.m && k0 + kk < ldbt) {
        breg[q] = *reinterpret_cast<const vt*>(Bt + (int64_t)(col0 + cc) * ldbt + k0 + kk);
      } else {
#pragma unroll
        for (int x = 0; x < W; ++x) breg[q][x] = T(0);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int e = q * NT + t;
      const int kk = e / ROWCH, rc = (e % ROWCH) * W;
      T* dst = &As[buf][kk * LDR + rc];
#pragma unroll
      for (int x = 0; x < W; ++x) {
        T v = areg[q][x];
        if constexpr (MODE == NN_ANALYSIS) v = (T)((double)v - mean[rc + x]);
        dst[x] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int e = q * NT + t;
      const int cc = e / BCH, kk = (e % BCH) * W;
#pragma unroll
      for (int x = 0; x < W; ++x) Bs[buf][(kk + x) * LDC + cc] = breg[q][x];
    }
  };

  int buf = 0;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int k0 = 0; k0 < p.K; k0 += KC) {
    const bool more = k0 + KC < p.K;
    if (more) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += MF::KSTEP) {
      T cop[CI], rop[RJ];
#pragma unroll
      for (int i = 0; i < CI; ++i) cop[i] = Bs[buf][(kk + l / 16) * LDC + c_off + 16 * i + l % 16];
#pragma unroll
      for (int j = 0; j < RJ; ++j) rop[j] = As[buf][(kk + l / 16) * LDR + r_off + 16 * j + l % 16];
#pragma unroll
      for (int i = 0; i < CI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = MF::mma(cop[i], rop[j], acc[i][j]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // acc[i][j] element (row = output column, col = output row)
  const T* __restrict__ Cin = static_cast<const T*>(p.Cin);
  T* __restrict__ Cout = static_cast<T*>(p.Cout);
#pragma unroll
  for (int i = 0; i < CI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j)
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

constexpr int64_t kTnTargetBlocks = 768;   // ~3 blocks per CU
constexpr int64_t kTnMinRows = 1024;

int64_t tn_chunks(int64_t n, int a, int m) {
  const int64_t tiles = (int64_t)((a + TILE - 1) / TILE) * ((m + TILE - 1) / TILE);
  int64_t chunks = (kTnTargetBlocks + tiles - 1) / tiles;
  const int64_t max_chunks = (n + kTnMinRows - 1) / kTnMinRows;
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
  const int tiles = ((a + TILE - 1) / TILE) * tiles_m;
  if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
  const size_t es = dt == ENKF_F64 ? 8 : 4;
  const bool vec = aligned16(A, lda, es) && aligned16(B, ldb, es);
  dim3 grid((unsigned)used, (unsigned)tiles);
  if (dt == ENKF_F64)
    tn_partial_kernel<double><<<grid, NT, 0, s>>>(n, a, m, (const double*)A, lda, (const double*)B, ldb, partial, rpc,
                                                  tiles_m, vec);
  else
    tn_partial_kernel<float><<<grid, NT, 0, s>>>(n, a, m, (const float*)A, lda, (const float*)B, ldb, partial, rpc,
                                                 tiles_m, vec);
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

int nn_bt_ld(int K) { return (K + 15) / 16 * 16; }

size_t nn_bt_bytes(int K, int m) { return sizeof(double) * (size_t)nn_bt_ld(K) * (size_t)m; }

namespace {

template <typename T, int MODE, int TR, int TC>
enkf_status nn_go(NnArgs p, const T* Bt, int ldbt, bool vec, hipStream_t s) {
  p.n_row_tiles = (p.n + TR - 1) / TR;
  p.n_col_tiles = (p.m + TC - 1) / TC;
  const int64_t groups = (p.n_row_tiles + 7) / 8;
  const int64_t blocks = groups * 8 * p.n_col_tiles;
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "nn product: grid too large");
  nn_kernel<T, MODE, TR, TC><<<(unsigned)blocks, NT, 0, s>>>(p, Bt, ldbt, vec);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

// Tile choice: one column tile of 128 when m <= 128 (64 rows), else
// 128 rows x 64 (FP64) or 128 (FP32) columns.
template <typename T, int MODE>
enkf_status nn_pick(NnArgs p, const T* Bt, int ldbt, bool vec, hipStream_t s) {
  if (p.m <= 128) return nn_go<T, MODE, 64, 128>(p, Bt, ldbt, vec, s);
  if constexpr (sizeof(T) == 8) return nn_go<T, MODE, 128, 64>(p, Bt, ldbt, vec, s);
  else return nn_go<T, MODE, 128, 128>(p, Bt, ldbt, vec, s);
}

template <typename T>
enkf_status nn_typed(int mode, NnArgs p, hipStream_t s) {
  T* Bt = static_cast<T*>(p.bws);
  const int ldbt = nn_bt_ld(p.K);
  const int64_t total = (int64_t)ldbt * p.m;
  convert_b_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(p.K, p.m, p.Bm, p.ldb, p.scale, Bt, ldbt);
  ENKF_HIP_CHECK(hipGetLastError());
  const bool vec = aligned16(p.A, p.lda, sizeof(T));
  if (mode == NN_UPDATE) return nn_pick<T, NN_UPDATE>(p, Bt, ldbt, vec, s);
  if (mode == NN_ANALYSIS) return nn_pick<T, NN_ANALYSIS>(p, Bt, ldbt, vec, s);
  return nn_pick<T, NN_RESIDUAL>(p, Bt, ldbt, vec, s);
}

}  // namespace

enkf_status launch_nn(enkf_dtype dt, int mode, NnArgs p, hipStream_t s) {
  if (p.n <= 0 || p.m <= 0) return ENKF_SUCCESS;
  if (!p.bws) return fail(ENKF_ERR_INVALID_ARG, "nn product: no workspace for the converted right factor");
  if (dt == ENKF_F64) return nn_typed<double>(mode, p, s);
  return nn_typed<float>(mode, p, s);
}

}  // namespace enkf
