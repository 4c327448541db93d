// Narrow-input matrix-core products of the mixed-precision blocked solve
// (gfx950, 16x16x32 MFMA with FP32 accumulation). Storage stays FP32; each
// operand is rounded when it is staged in LDS:
//   BF16    x -> bf16(x)
//   F16     x -> f16(x)
//   BF16X3  x -> hi + mid + lo, three bf16 (~24 significant bits); a product
//           takes the six cross products down to 2^-24 (six passes)
//   F16X2   x -> hi + lo/2^11, hi = f16(x), lo = f16((x - hi) 2^11); the
//           cross terms go to a second accumulator scaled by 2^-11 at the end
// Same two products as gemm_mfma.hip, with the same pipeline (branch-free
// register prefetch of the next stage kept ahead of the matrix-core work):
//   tn: P = A^T B over n rows, split-K partials (FP64), fixed-order sum;
//   nn: X <- X - A Bm (UPDATE) and XA <- XB + (XB - xbar 1^T)(s Bm) (ANALYSIS);
//       the right factor is split into its narrow parts once per call.
#include <atomic>

#include "enkf_internal.h"
#include "gemm_lowp.h"
#include "gemm_mfma.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int NT = 256;
constexpr int TILE = 128;
constexpr int KC = 32;             // one 16x16x32 step per stage
constexpr int LDK = KC + 8;        // 16-bit elements; keeps 16-byte alignment

// Split policy: an FP32 value becomes PARTS narrow values; a product sums
// NPROD part-by-part MFMAs (pa[q], pb[q]); products with scaled[q] go to a
// second accumulator multiplied by 2^-11 at the end (FP16 low parts are
// stored scaled by 2^11 to stay in range).
template <int MATH> struct Lp;
template <> struct Lp<ENKF_MATH_BF16> {
  typedef __bf16 e_t;
  typedef mf_bf8 v_t;
  static constexpr int PARTS = 1, NPROD = 1;
  static constexpr bool has_scaled = false;
  static __device__ __forceinline__ void conv(float x, e_t* o) { o[0] = (__bf16)x; }
  static __device__ __forceinline__ mf_f4 mma(v_t a, v_t b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Lp<ENKF_MATH_F16> {
  typedef _Float16 e_t;
  typedef mf_h8 v_t;
  static constexpr int PARTS = 1, NPROD = 1;
  static constexpr bool has_scaled = false;
  static __device__ __forceinline__ void conv(float x, e_t* o) { o[0] = (_Float16)x; }
  static __device__ __forceinline__ mf_f4 mma(v_t a, v_t b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
// x = hi + mid + lo (three bf16, ~24 significant bits); six products
// hi*hi + hi*mid + mid*hi + hi*lo + mid*mid + lo*hi (terms below 2^-24 dropped).
template <> struct Lp<ENKF_MATH_BF16X3> {
  typedef __bf16 e_t;
  typedef mf_bf8 v_t;
  static constexpr int PARTS = 3, NPROD = 6;
  static constexpr bool has_scaled = false;
  static __device__ __forceinline__ void conv(float x, e_t* o) {
    o[0] = (__bf16)x;
    const float r1 = x - (float)o[0];
    o[1] = (__bf16)r1;
    o[2] = (__bf16)(r1 - (float)o[1]);
  }
  static __device__ __forceinline__ mf_f4 mma(v_t a, v_t b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
// x = hi + lo 2^-11 (two f16, ~22 bits); hi*hi + (hi*lo + lo*hi) 2^-11.
template <> struct Lp<ENKF_MATH_F16X2> {
  typedef _Float16 e_t;
  typedef mf_h8 v_t;
  static constexpr int PARTS = 2, NPROD = 3;
  static constexpr bool has_scaled = true;
  static __device__ __forceinline__ void conv(float x, e_t* o) {
    o[0] = (_Float16)x;
    o[1] = (_Float16)((x - (float)o[0]) * 2048.f);
  }
  static __device__ __forceinline__ mf_f4 mma(v_t a, v_t b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
// product q multiplies part PA[q] of the first operand by part PB[q] of the second
__device__ constexpr int kPA[6] = {0, 0, 1, 0, 1, 2};
__device__ constexpr int kPB[6] = {0, 1, 0, 2, 1, 0};
constexpr float kLoScale = 1.0f / 2048.f;

template <typename V>
__device__ __forceinline__ V ld8(const void* p) {
  return *reinterpret_cast<const V*>(p);
}

typedef float f4v __attribute__((ext_vector_type(4)));

// Branch-free staged loads (as in gemm_mfma.hip): an index outside the valid
// range reads a valid element; values that matter are zeroed when staged.
template <bool VEC>
__device__ __forceinline__ f4v load4(const float* __restrict__ col, int64_t row, int64_t rlim) {
  f4v v;
  if constexpr (VEC) {
    v = *reinterpret_cast<const f4v*>(col + (row < rlim ? row : 0));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = col[row + e < rlim ? row + e : 0];
  }
  return v;
}

// ---------------------------------------------------------------- tn
// Stage layout: S[q][col][k] per part q, col in [0, TA + TILE): A columns
// then B columns; k contiguous (LDK), so an MFMA operand is one 16-byte read.
// 4 waves, 2 (m) x 2 (a); wave tile 64 x 32 (4 x 2 MFMA tiles); block tile
// 128 (m) x 64 (a). FP32 accumulators are emptied into FP64 every kFlush
// stages (one-pass forms: their own rounding dominates, so less often).
constexpr int TA = 64;

template <int MATH, bool VEC>
__global__ __launch_bounds__(NT, 2) void tn_lowp_kernel(int64_t n, int a, int m, const float* __restrict__ A,
                                                        int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                        double* __restrict__ partial, int64_t rows_per_chunk,
                                                        int tiles_m) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  typedef typename P::v_t VT;
  constexpr int COLS = TA + TILE;
  constexpr int PER_COL = KC / 4;
  constexpr int COLS_PER_PASS = NT / PER_COL;
  constexpr int PASSES = COLS / COLS_PER_PASS;
  constexpr int kFlush = P::PARTS == 1 ? 8 : 2;
  __shared__ __attribute__((aligned(16))) E S[P::PARTS][COLS * LDK];

  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * TA, m0 = tm * TILE;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int m_off = (w / 2) * 64, a_off = (w % 2) * 32;
  const int lc = t / PER_COL, lk = (t % PER_COL) * 4;
  const float* cp[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const int c = p * COLS_PER_PASS + lc;
    if (c < TA) cp[p] = A + (int64_t)min(a0 + c, a - 1) * lda;
    else cp[p] = B + (int64_t)min(m0 + c - TA, m - 1) * ldb;
  }
  mf_f4 acc[4][2], acc2[P::has_scaled ? 4 : 1][P::has_scaled ? 2 : 1];
  double wide[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (P::has_scaled) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) wide[i][j][r] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = (double)acc[i][j][r];
          if constexpr (P::has_scaled) v += (double)acc2[i][j][r] * (double)kLoScale;
          wide[i][j][r] += v;
        }
        acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (P::has_scaled) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  f4v reg[PASSES];
  auto fetch = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) reg[p] = load4<VEC>(cp[p], rs + lk, r1);
  };
  auto stash = [&](int64_t rs) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int o = (p * COLS_PER_PASS + lc) * LDK + lk;
      E parts[4][P::PARTS];
#pragma unroll
      for (int e = 0; e < 4; ++e) P::conv(rs + lk + e < r1 ? reg[p][e] : 0.f, parts[e]);
#pragma unroll
      for (int q = 0; q < P::PARTS; ++q) {
        typedef E e4 __attribute__((ext_vector_type(4)));
        e4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = parts[e][q];
        *reinterpret_cast<e4*>(&S[q][o]) = v;
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
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int pr = 0; pr < P::NPROD; ++pr) {
      const int pa = kPA[pr], pb = kPB[pr];
      VT bo[4], ao[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) bo[i] = ld8<VT>(&S[pa][(TA + m_off + 16 * i + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int j = 0; j < 2; ++j) ao[j] = ld8<VT>(&S[pb][(a_off + 16 * j + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (P::has_scaled && pr > 0) acc2[i][j] = P::mma(bo[i], ao[j], acc2[i][j]);
          else acc[i][j] = P::mma(bo[i], ao[j], acc[i][j]);
        }
    }
    if (++stage == kFlush) {
      flush();
      stage = 0;
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(rs + KC);
    __syncthreads();
  }
  flush();
  double* Pp = partial + (int64_t)blockIdx.x * a * m;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mi = m0 + m_off + 16 * i + 4 * (l / 16) + r;
        const int ai = a0 + a_off + 16 * j + l % 16;
        if (mi < m && ai < a) Pp[ai + (int64_t)mi * a] = wide[i][j][r];
      }
}

// ---------------------------------------------------------------- nn
// The right factor scale * Bm is split into parts once per call:
// Bp[q][col * ldk + k], ldk = nn_bt_rows(K) (zero past K), columns padded to
// nn_bt_cols(m) (zero past m).
template <int MATH>
__global__ __launch_bounds__(256) void split_b_kernel(int K, int m, const double* __restrict__ Bm, int64_t ldb,
                                                      double scale, typename Lp<MATH>::e_t* __restrict__ Bp, int ldk,
                                                      int cols) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)ldk * cols;
  if (e >= total) return;
  const int k = (int)(e % ldk), j = (int)(e / ldk);
  const float x = (k < K && j < m) ? (float)(scale * Bm[k + (int64_t)j * ldb]) : 0.f;
  E parts[P::PARTS];
  P::conv(x, parts);
#pragma unroll
  for (int q = 0; q < P::PARTS; ++q) Bp[q * total + e] = parts[q];
}

// Stage layout: As[q][row][k], Bs[q][col][k] (k contiguous, LDK). A items:
// 4 rows x 4 k (four 16-byte column loads, four 8-byte LDS writes per part);
// B items: 8 k of one column (one 16-byte load and write per part).
// 4 waves, 2 x 2: wave (w/2, w%2) owns TC/2 columns x TR/2 rows.
template <int MATH, int MODE, int TR, int TC, bool VEC, bool LOOP>
__global__ __launch_bounds__(NT, 2) void nn_lowp_kernel(NnArgs p, const typename Lp<MATH>::e_t* __restrict__ Bp,
                                                        int ldk, int64_t bp_stride) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  typedef typename P::v_t VT;
  constexpr int CI = TC / 32, RJ = TR / 32;
  constexpr int KE = TR * KC / (4 * NT);           // k per A item (4 rows x KE k)
  static_assert(KE == 2 || KE == 4, "A item shape");
  constexpr int A_ITEMS = (TR / 4) * (KC / KE);
  constexpr int A_PASSES = A_ITEMS / NT;
  constexpr int B_ITEMS = TC * (KC / 8);
  constexpr int B_PASSES = B_ITEMS / NT;
  static_assert(A_PASSES >= 1 && B_PASSES >= 1, "tile too small for the block");
  __shared__ __attribute__((aligned(16))) E As[P::PARTS][TR * LDK];
  __shared__ __attribute__((aligned(16))) E Bs[P::PARTS][TC * LDK];
  __shared__ double mean[TR];
  int64_t rt;
  int ct;
  // LOOP: one block takes every column tile of its row tile (the row means of
  // ANALYSIS are then formed once per row tile). It is a separate instance so
  // that one-tile launches keep their register budget (occupancy).
  static_assert(!LOOP || MODE == NN_ANALYSIS, "only ANALYSIS walks the column tiles");
  xcd_tile_map(blockIdx.x, p.n_row_tiles, LOOP ? 1 : p.n_col_tiles, &rt, &ct);
  if (rt >= p.n_row_tiles) return;
  const int64_t row0 = rt * TR;
  const float* __restrict__ A = static_cast<const float*>(p.A);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int c_off = (w / 2) * (TC / 2), r_off = (w % 2) * (TR / 2);
  const int64_t rlim = p.n;
  if constexpr (MODE == NN_ANALYSIS) {
    constexpr int Q = NT / TR;
    constexpr int U = 8;
    __shared__ double part[Q][TR];
    const int rr = t % TR, q = t / TR;
    const float* __restrict__ ar = A + min(row0 + rr, rlim - 1);
    double s = 0.0;
    int j = q;
    for (; j + (U - 1) * Q < p.K; j += U * Q) {
      float x[U];
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
  mf_f4 acc[CI][RJ], acc2[P::has_scaled ? CI : 1][P::has_scaled ? RJ : 1];
#pragma unroll
  for (int i = 0; i < CI; ++i)
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (P::has_scaled) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
    }

  f4v areg[A_PASSES][KE];
  VT breg[B_PASSES][P::PARTS];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int it = q * NT + t;
      const int rq = (it % (TR / 4)) * 4, kq = (it / (TR / 4)) * KE;
#pragma unroll
      for (int e = 0; e < KE; ++e) {
        const int k = min(k0 + kq + e, p.K - 1);
        areg[q][e] = load4<VEC>(A + (int64_t)k * p.lda, row0 + rq, rlim);
      }
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int it = q * NT + t;
      const int cc = it % TC, kg = (it / TC) * 8;
      const int k = min(k0 + kg, ldk - 8);
#pragma unroll
      for (int z = 0; z < P::PARTS; ++z)
        breg[q][z] = ld8<VT>(Bp + z * bp_stride + (int64_t)(col0 + cc) * ldk + k);
    }
  };
  auto stash = [&](int k0) {
#pragma unroll
    for (int q = 0; q < A_PASSES; ++q) {
      const int it = q * NT + t;
      const int rq = (it % (TR / 4)) * 4, kq = (it / (TR / 4)) * KE;
      // element (row rq + x, k kq + e) = areg[q][e][x]
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        E parts[KE][P::PARTS];
#pragma unroll
        for (int e = 0; e < KE; ++e) {
          float v = areg[q][e][x];
          if constexpr (MODE == NN_ANALYSIS) v = (float)((double)v - mean[rq + x]);
          P::conv(k0 + kq + e < p.K ? v : 0.f, parts[e]);
        }
#pragma unroll
        for (int z = 0; z < P::PARTS; ++z) {
          typedef E ek __attribute__((ext_vector_type(KE)));
          ek vk;
#pragma unroll
          for (int e = 0; e < KE; ++e) vk[e] = parts[e][z];
          *reinterpret_cast<ek*>(&As[z][(rq + x) * LDK + kq]) = vk;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < B_PASSES; ++q) {
      const int it = q * NT + t;
      const int cc = it % TC, kg = (it / TC) * 8;
#pragma unroll
      for (int z = 0; z < P::PARTS; ++z) *reinterpret_cast<VT*>(&Bs[z][cc * LDK + kg]) = breg[q][z];
    }
  };

  fetch(0);
  stash(0);
  __syncthreads();
  for (int k0 = 0; k0 < p.K; k0 += KC) {
    fetch(k0 + KC);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int pr = 0; pr < P::NPROD; ++pr) {
      const int pa = kPA[pr], pb = kPB[pr];
      VT co[CI], ro[RJ];
#pragma unroll
      for (int i = 0; i < CI; ++i) co[i] = ld8<VT>(&Bs[pa][(c_off + 16 * i + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int j = 0; j < RJ; ++j) ro[j] = ld8<VT>(&As[pb][(r_off + 16 * j + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int i = 0; i < CI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) {
          if (P::has_scaled && pr > 0) acc2[i][j] = P::mma(co[i], ro[j], acc2[i][j]);
          else acc[i][j] = P::mma(co[i], ro[j], acc[i][j]);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(k0 + KC);
    __syncthreads();
  }
  // epilogue: inputs loaded first (clamped, branch-free), stores predicated
  float* __restrict__ Cout = static_cast<float*>(p.Cout);
  const float* __restrict__ Cin = static_cast<const float*>(p.Cin);
  double zsc = 1.0;                               // UPDATE64: the FP16 forms' rms scale
  if constexpr (MODE == NN_UPDATE64) zsc = rms_scale(p.z64_sumsq, (double)p.n * p.m);
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    float cin[RJ][4];
    double zin[RJ][4];                            // UPDATE64: the FP64 destination's values (when it accumulates)
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int64_t row = min(row0 + r_off + 16 * j + l % 16, rlim - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = min(col0 + c_off + 16 * i + 4 * (l / 16) + r, p.m - 1);
        cin[j][r] = Cin[row + (int64_t)col * p.ldc];
        if constexpr (MODE == NN_UPDATE64) zin[j][r] = p.z64_acc ? p.Z64[row + (int64_t)col * p.ldz64] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < RJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + c_off + 16 * i + 4 * (l / 16) + r;
        const int64_t row = row0 + r_off + 16 * j + l % 16;
        double prod = (double)acc[i][j][r];
        if constexpr (P::has_scaled) prod += (double)acc2[i][j][r] * (double)kLoScale;
        const double c = (double)cin[j][r];
        const double out = (MODE == NN_ANALYSIS) ? c + prod : c - prod;
        if constexpr (MODE == NN_UPDATE64) {
          if (col < p.m && row < p.n)
            p.Z64[row + (int64_t)col * p.ldz64] = zin[j][r] + zsc * out;
        } else {
          if (col < p.m && row < p.n) Cout[row + (int64_t)col * p.ldo] = (float)out;
        }
      }
  }
  }
}

// ---------------------------------------------------------------- analysis, row tile resident
// X^A = X^B + (X^B - xbar 1^T) (s G) with one-pass 16-bit inputs (BF16 or
// F16), K = N <= kResMaxK and X^A's columns the members (m = K): X^B is read
// from memory once and X^A written once. A block owns 64 rows; wave w owns
// the members (= output columns) [128 w, 128 w + 128) and loads them into
// registers, lane (a, b) = (l % 16, l / 16) taking rows 4a .. 4a + 3 of the
// 32 members 128 w + 32 b + z (16-byte loads, 256 contiguous bytes of a
// column per 16 lanes). The row means are reduced across lanes and waves;
// the centred rows, rounded to the input type, go to the LDS as the MFMA's
// row operand, resident for every output column. Each wave then forms its
// 64 x 128 output as two groups of 4 x 4 MFMA tiles of 16 x 16 over K, the
// right factor's fragments streamed from the L2 (fragment-ordered, 1 KB per
// wave load, a two-stage register ring). The accumulators go through a small
// per-wave LDS buffer, 8 columns at a time, back to the load layout, where
// the registers still hold X^B for the sum, and X^A leaves in 256-byte
// column runs again. The right factor's columns are permuted (see
// res_frag_index) so that an MFMA tile's half holds exactly the 8 columns
// the load layout needs next.
constexpr int RT_ROWS = 64;
constexpr int RT_CPW = 128;                // members per wave
constexpr int RT_MAXW = 8;
constexpr int kResMaxK = RT_CPW * RT_MAXW;
constexpr int RT_TCOLS = 8;                // columns per transpose piece
constexpr int RT_TLD = RT_ROWS + 4;        // column stride (floats) of a transpose buffer: spreads the banks

// Position of the right factor's element (k, c) in the fragment-ordered copy.
// Column c: wave w = c / 128, u = c % 128 = 32 b + 2 pi + d (the load layout:
// lane quarter b, piece pi in [0, 16), d in {0, 1}); piece pi = 8 h + 2 i + e
// is half e of MFMA column tile i of group h, whose lane p = 8 e + 2 b + d.
// Fragment (tile T = 8 w + 4 h + i, k chunk kc) is 512 elements, lane l's 8
// values (k = 32 kc + 8 (l / 16) + 0..7, column slot l % 16) contiguous.
__device__ __forceinline__ int64_t res_frag_index(int k, int c, int nkc) {
  const int w = c / RT_CPW, u = c % RT_CPW;
  const int b = u / 32, z = u % 32, pi = z / 2, d = z % 2;
  const int h = pi / 8, i = (pi % 8) / 2, e = pi % 2;
  const int pl = 8 * e + 2 * b + d;
  const int64_t tile = 8 * w + 4 * h + i;
  return ((tile * nkc + k / 32) * 64 + 16 * ((k % 32) / 8) + pl) * 8 + k % 8;
}

template <int MATH>
__global__ __launch_bounds__(256) void split_res_kernel(int K, int m, const double* __restrict__ Bm, int64_t ldb,
                                                        double scale, typename Lp<MATH>::e_t* __restrict__ Bf, int kp,
                                                        int ncols) {
  typedef typename Lp<MATH>::e_t E;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kp * ncols) return;
  const int k = (int)(e % kp), c = (int)(e / kp);
  const float x = (k < K && c < m) ? (float)(scale * Bm[k + (int64_t)c * ldb]) : 0.f;
  E part[1];
  Lp<MATH>::conv(x, part);
  Bf[res_frag_index(k, c, kp / 32)] = part[0];
}

template <int MATH>
__global__ __launch_bounds__(64 * RT_MAXW, 1) void analysis_res_kernel(NnArgs p, const typename Lp<MATH>::e_t* __restrict__ Bf,
                                                                      int kp) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  typedef typename P::v_t VT;
  static_assert(P::PARTS == 1, "one-pass inputs only");
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  __shared__ double red[RT_MAXW][RT_ROWS];
  __shared__ double mean[RT_ROWS];
  const int K = p.K, nw = blockDim.x / kWave;
  const int lds_ld = kp + 8;                       // tile row stride in elements
  E* As = reinterpret_cast<E*>(lds_raw);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  float* tb = reinterpret_cast<float*>(lds_raw + (size_t)RT_ROWS * lds_ld * sizeof(E)) + w * RT_TCOLS * RT_TLD;
  const int a = l % 16, b = l / 16;                // load layout
  const int pq = l % 16, q = l / 16;               // MFMA layout
  const int64_t row0 = (int64_t)blockIdx.x * RT_ROWS;
  const int64_t r4 = row0 + 4 * a;
  const int cw = RT_CPW * w + 32 * b;              // this lane's first member
  const float* __restrict__ A = static_cast<const float*>(p.A);
  float* __restrict__ Cout = static_cast<float*>(p.Cout);
  const bool vin = ((uintptr_t)A % 16) == 0 && (p.lda % 4) == 0 && r4 + 3 < p.n;
  const bool vout = ((uintptr_t)Cout % 16) == 0 && (p.ldo % 4) == 0 && r4 + 3 < p.n;
  // 1. X^B rows 4a .. + 3, members cw .. cw + 31 (clamped past K and n; those are never used)
  f4v xs[32];
#pragma unroll
  for (int z = 0; z < 32; ++z) {
    const float* col = A + (int64_t)min(cw + z, K - 1) * p.lda;
    if (vin) {
      xs[z] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(col + r4));
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) xs[z][e] = col[min(r4 + e, p.n - 1)];
    }
  }
  // 2. row means in FP64: lane sums, then over the four lane quarters, then over the waves
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int z = 0; z < 32; ++z)
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += cw + z < K ? (double)xs[z][e] : 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    s[e] += __shfl_xor(s[e], 16);
    s[e] += __shfl_xor(s[e], 32);
  }
  if (b == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) red[w][4 * a + e] = s[e];
  }
  __syncthreads();
  if (t < RT_ROWS) {
    double tot = 0.0;
    for (int z = 0; z < nw; ++z) tot += red[z][t];
    mean[t] = tot / (double)K;
  }
  __syncthreads();
  // 3. the centred tile, rounded to the input type (the FP64 mean split into
  //    two floats: x - mean to FP32 accuracy); members past K are zero
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double mu = mean[4 * a + e];
    const float mh = (float)mu, ml = (float)(mu - (double)mh);
#pragma unroll
    for (int c8 = 0; c8 < 4; ++c8) {
      const int k0 = cw + 8 * c8;
      if (k0 < kp) {
        VT v;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          E part[1];
          P::conv(k0 + u < K ? (xs[8 * c8 + u][e] - mh) - ml : 0.f, part);
          v[u] = part[0];
        }
        *reinterpret_cast<VT*>(&As[(4 * a + e) * lds_ld + k0]) = v;
      }
    }
  }
  __syncthreads();
  // 4. products, two groups of 64 columns, and the epilogue through tb
  const E* arow[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) arow[j] = As + (16 * j + pq) * lds_ld + 8 * q;
  const int nkc = kp / 32;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    mf_f4 acc[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[j][i] = mf_f4{0.f, 0.f, 0.f, 0.f};
    const E* bb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bb[i] = Bf + (int64_t)(8 * w + 4 * h + i) * nkc * 512 + l * 8;
    VT bq[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bq[0][i] = ld8<VT>(bb[i]);
      bq[1][i] = ld8<VT>(bb[i] + 512 * min(1, nkc - 1));
    }
    for (int kc = 0; kc < nkc; kc += 2) {
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        if (kc + st < nkc) {                       // nkc odd: the second stage of the last pair is empty
          VT ro[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) ro[j] = ld8<VT>(arow[j] + 32 * (kc + st));
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[j][i] = P::mma(ro[j], bq[st][i], acc[j][i]);
          // the chunk two ahead (past the end: the last chunk again, unused)
#pragma unroll
          for (int i = 0; i < 4; ++i) bq[st][i] = ld8<VT>(bb[i] + 512 * min(kc + st + 2, nkc - 1));
        }
      }
    }
    // acc[j][i] element r: row 16 j + 4 q + r, column slot (h, i, pq): member
    // cw' + 2 pi + d of lane quarter b' with pq = 8 e + 2 b' + d, pi = 8 h + 2 i + e
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int pi = 8 * h + 2 * i + e;
        if (pq / 8 == e) {
#pragma unroll
          for (int j = 0; j < 4; ++j) *reinterpret_cast<mf_f4*>(&tb[(pq % 8) * RT_TLD + 16 * j + 4 * q]) = acc[j][i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const f4v v = *reinterpret_cast<const f4v*>(&tb[(2 * b + d) * RT_TLD + 4 * a]);
          const int c = cw + 2 * pi + d;
          f4v o;
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) o[e2] = (float)((double)xs[2 * pi + d][e2] + (double)v[e2]);
          if (c < p.m) {
            float* dst = Cout + (int64_t)c * p.ldo;
            if (vout) {
              __builtin_nontemporal_store(o, reinterpret_cast<f4v*>(dst + r4));
            } else {
#pragma unroll
              for (int e2 = 0; e2 < 4; ++e2)
                if (r4 + e2 < p.n) dst[r4 + e2] = o[e2];
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
  }
}

template <int MATH>
enkf_status analysis_res_go(const NnArgs& p, hipStream_t s) {
  typedef typename Lp<MATH>::e_t E;
  E* Bf = static_cast<E*>(p.bws);
  const int kp = (p.K + 31) / 32 * 32;
  const int nw = (p.K + RT_CPW - 1) / RT_CPW, ncols = nw * RT_CPW;
  const int64_t total = (int64_t)kp * ncols;
  split_res_kernel<MATH><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(p.K, p.m, p.Bm, p.ldb, p.scale, Bf, kp, ncols);
  ENKF_HIP_CHECK(hipGetLastError());
  const size_t lds = (size_t)RT_ROWS * (kp + 8) * sizeof(E) + (size_t)nw * RT_TCOLS * RT_TLD * sizeof(float);
  static std::atomic<uint64_t> attr{0};
  const size_t most = (size_t)RT_ROWS * (kResMaxK + 8) * sizeof(E) + (size_t)RT_MAXW * RT_TCOLS * RT_TLD * sizeof(float);
  enkf_status st = set_dynamic_lds(attr, (const void*)analysis_res_kernel<MATH>, most,
                                   "analysis product: cannot set the LDS size");
  if (st != ENKF_SUCCESS) return st;
  const int64_t blocks = (p.n + RT_ROWS - 1) / RT_ROWS;
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "analysis product: too many rows for the grid");
  analysis_res_kernel<MATH><<<(unsigned)blocks, kWave * nw, lds, s>>>(p, Bf, kp);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

template <int MATH>
void tn_launch(dim3 grid, hipStream_t s, int64_t n, int a, int m, const float* A, int64_t lda, const float* B,
               int64_t ldb, double* partial, int64_t rpc, int tiles_m, bool vec) {
  if (vec) tn_lowp_kernel<MATH, true><<<grid, NT, 0, s>>>(n, a, m, A, lda, B, ldb, partial, rpc, tiles_m);
  else tn_lowp_kernel<MATH, false><<<grid, NT, 0, s>>>(n, a, m, A, lda, B, ldb, partial, rpc, tiles_m);
}

template <int MATH, int MODE, int TR, int TC>
void nn_go(NnArgs p, const typename Lp<MATH>::e_t* Bp, int ldk, int64_t stride, bool vec, hipStream_t s) {
  p.n_row_tiles = (p.n + TR - 1) / TR;
  p.n_col_tiles = (p.m + TC - 1) / TC;
  // ANALYSIS with several column tiles and rows enough to fill the part: one
  // block per row tile walks its column tiles (row means formed once)
  // the walk over column tiles only where its instance keeps every register
  // (vector loads; the two-part FP16 split would spill)
  constexpr bool kLoopable = MODE == NN_ANALYSIS && TR == 128 && MATH != ENKF_MATH_F16X2;
  const bool loop = kLoopable && vec && p.n_col_tiles > 1 && p.n_row_tiles >= 2048;
  const int64_t groups = (p.n_row_tiles + 7) / 8;
  const unsigned g = (unsigned)(groups * 8 * (loop ? 1 : p.n_col_tiles));
  if constexpr (kLoopable) {
    if (loop) {
      nn_lowp_kernel<MATH, MODE, TR, TC, true, true><<<g, NT, 0, s>>>(p, Bp, ldk, stride);
      return;
    }
  }
  if (vec) nn_lowp_kernel<MATH, MODE, TR, TC, true, false><<<g, NT, 0, s>>>(p, Bp, ldk, stride);
  else nn_lowp_kernel<MATH, MODE, TR, TC, false, false><<<g, NT, 0, s>>>(p, Bp, ldk, stride);
}

template <int MATH>
enkf_status nn_launch(hipStream_t s, int mode, NnArgs p) {
  typedef typename Lp<MATH>::e_t E;
  E* Bp = static_cast<E*>(p.bws);
  const int ldk = nn_bt_rows(p.K), cols = nn_bt_cols(p.m);
  const int64_t stride = (int64_t)ldk * cols;
  if constexpr (Lp<MATH>::PARTS == 1) {
    // the analysis with many rows: X^B read once, the row tile resident in
    // the LDS for every output column (the tiled kernel re-reads it per
    // column tile and reads X^B again for the sum)
    if (mode == NN_ANALYSIS && p.K <= kResMaxK && p.m == p.K && p.n >= 64 * 1024 && p.Cin == p.A &&
        p.ldc == p.lda)
      return analysis_res_go<MATH>(p, s);
  }
  split_b_kernel<MATH><<<(unsigned)((stride + 255) / 256), 256, 0, s>>>(p.K, p.m, p.Bm, p.ldb, p.scale, Bp, ldk, cols);
  ENKF_HIP_CHECK(hipGetLastError());
  const int64_t rows = (p.n + 63) / 64;
  if ((p.m <= 128 ? rows : (p.n + 127) / 128) * 8 * ((p.m + 127) / 128) > 0x7fffffff)
    return fail(ENKF_ERR_NOT_SUPPORTED, "nn product: grid too large");
  const bool vec = ((uintptr_t)p.A % 16) == 0 && (p.lda % 4) == 0 && (p.n % 4) == 0;
  if (mode == NN_UPDATE64) {
    // the last panel update of a mixed solve into the FP64 solution
    if (!p.Z64) return fail(ENKF_ERR_INVALID_ARG, "update product: no FP64 destination");
    if (p.m <= 128) nn_go<MATH, NN_UPDATE64, 64, 128>(p, Bp, ldk, stride, vec, s);
    else nn_go<MATH, NN_UPDATE64, 128, 128>(p, Bp, ldk, stride, vec, s);
    ENKF_HIP_CHECK(hipGetLastError());
    return ENKF_SUCCESS;
  }
  if (p.m <= 128) {
    if (mode == NN_ANALYSIS) nn_go<MATH, NN_ANALYSIS, 64, 128>(p, Bp, ldk, stride, vec, s);
    else nn_go<MATH, NN_UPDATE, 64, 128>(p, Bp, ldk, stride, vec, s);
  } else {
    if (mode == NN_ANALYSIS) nn_go<MATH, NN_ANALYSIS, 128, 128>(p, Bp, ldk, stride, vec, s);
    else nn_go<MATH, NN_UPDATE, 128, 128>(p, Bp, ldk, stride, vec, s);
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace

enkf_status launch_tn_lowp(enkf_math math, int64_t n, int a, int m, const float* A, int64_t lda, const float* B,
                           int64_t ldb, double* G, int64_t ldg, double* partial, hipStream_t s) {
  if (a <= 0 || m <= 0) return ENKF_SUCCESS;
  const int64_t chunks = tn_partial_elems(n, a, m) / ((int64_t)a * m);
  int64_t rpc = (n + chunks - 1) / chunks;
  rpc = ((rpc + KC - 1) / KC) * KC;
  const int64_t used = (n + rpc - 1) / rpc;
  const int tiles_m = (m + TILE - 1) / TILE;
  const int tiles = ((a + TA - 1) / TA) * tiles_m;
  if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
  const bool vec = ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0 && (lda % 4) == 0 && (ldb % 4) == 0 &&
                   (n % 4) == 0;
  dim3 grid((unsigned)used, (unsigned)tiles);
  switch (math) {
    case ENKF_MATH_BF16: tn_launch<ENKF_MATH_BF16>(grid, s, n, a, m, A, lda, B, ldb, partial, rpc, tiles_m, vec); break;
    case ENKF_MATH_F16: tn_launch<ENKF_MATH_F16>(grid, s, n, a, m, A, lda, B, ldb, partial, rpc, tiles_m, vec); break;
    case ENKF_MATH_BF16X3:
      tn_launch<ENKF_MATH_BF16X3>(grid, s, n, a, m, A, lda, B, ldb, partial, rpc, tiles_m, vec);
      break;
    case ENKF_MATH_F16X2: tn_launch<ENKF_MATH_F16X2>(grid, s, n, a, m, A, lda, B, ldb, partial, rpc, tiles_m, vec); break;
    default: return fail(ENKF_ERR_INVALID_ARG, "tn product: not a narrow math type");
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return launch_partial_sum(a, m, used, partial, G, ldg, s);
}

enkf_status launch_nn_lowp(enkf_math math, int mode, NnArgs p, hipStream_t s) {
  if (p.n <= 0 || p.m <= 0) return ENKF_SUCCESS;
  if (mode == NN_RESIDUAL) return fail(ENKF_ERR_NOT_SUPPORTED, "the residual is formed in FP64");
  if (!p.bws) return fail(ENKF_ERR_INVALID_ARG, "nn product: no workspace for the split right factor");
  switch (math) {
    case ENKF_MATH_BF16: return nn_launch<ENKF_MATH_BF16>(s, mode, p);
    case ENKF_MATH_F16: return nn_launch<ENKF_MATH_F16>(s, mode, p);
    case ENKF_MATH_BF16X3: return nn_launch<ENKF_MATH_BF16X3>(s, mode, p);
    case ENKF_MATH_F16X2: return nn_launch<ENKF_MATH_F16X2>(s, mode, p);
    default: return fail(ENKF_ERR_INVALID_ARG, "nn product: not a narrow math type");
  }
}

}  // namespace enkf
