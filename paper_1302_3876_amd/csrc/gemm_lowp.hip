// Narrow-input matrix-core products of the mixed-precision blocked solve
// (gfx950, 16x16x32 MFMA with FP32 accumulation). Storage stays FP32; each
// operand is rounded when it is staged in LDS:
//   BF16    x -> bf16(x)
//   F16     x -> f16(x)
//   BF16X3  x -> hi + mid + lo, three bf16 (~24 significant bits); a product
//           takes the six cross products down to 2^-24 (six passes)
//   F16X2   x -> hi + lo/2^11, hi = f16(x), lo = f16((x - hi) 2^11); the
//           cross terms go to a second accumulator scaled by 2^-11 at the end
// Same two products as gemm_mfma.hip:
//   tn: P = A^T B over n rows, split-K partials (FP64), fixed-order sum;
//   nn: X <- X - A Bm (UPDATE) and XA <- XB + (XB - xbar 1^T)(s Bm) (ANALYSIS).
// FP32 accumulators are emptied into FP64 every stage of rows (tn).
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

// ---------------------------------------------------------------- tn
// Stage layout: hi/lo[col][k], col in [0, 2*TILE): A columns then B columns.
template <int MATH>
__global__ __launch_bounds__(NT) void tn_lowp_kernel(int64_t n, int a, int m, const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ B, int64_t ldb,
                                                     double* __restrict__ partial, int64_t rows_per_chunk, int tiles_m,
                                                     bool vec) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  typedef typename P::v_t VT;
  typedef float f4v __attribute__((ext_vector_type(4)));
  constexpr int COLS = 2 * TILE;
  constexpr int PER_COL = KC / 4;
  constexpr int COLS_PER_PASS = NT / PER_COL;
  constexpr int PASSES = COLS / COLS_PER_PASS;
  __shared__ __attribute__((aligned(16))) E S[P::PARTS][COLS * LDK];

  const int ta = blockIdx.y / tiles_m, tm = blockIdx.y % tiles_m;
  const int a0 = ta * TILE, m0 = tm * TILE;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(n, r0 + rows_per_chunk);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int m_off = (w / 2) * 64, a_off = (w % 2) * 64;
  const int lc = t / PER_COL, lk = (t % PER_COL) * 4;
  const float* cp[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    const int c = p * COLS_PER_PASS + lc;
    if (c < TILE) cp[p] = (a0 + c < a) ? A + (int64_t)(a0 + c) * lda : nullptr;
    else cp[p] = (m0 + c - TILE < m) ? B + (int64_t)(m0 + c - TILE) * ldb : nullptr;
  }
  mf_f4 acc[4][4], acc2[P::has_scaled ? 4 : 1][P::has_scaled ? 4 : 1];
  double wide[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) wide[i][j][r] = 0.0;
    }
  if constexpr (P::has_scaled) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
  }
  f4v reg[PASSES];
  for (int64_t rs = r0; rs < r1; rs += KC) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (cp[p]) {
        const int64_t row = rs + lk;
        if (vec && row + 4 <= r1) v = *reinterpret_cast<const f4v*>(cp[p] + row);
        else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (row + e < r1) ? cp[p][row + e] : 0.f;
        }
      }
      reg[p] = v;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int o = (p * COLS_PER_PASS + lc) * LDK + lk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        E parts[P::PARTS];
        P::conv(reg[p][e], parts);
#pragma unroll
        for (int q = 0; q < P::PARTS; ++q) S[q][o + e] = parts[q];
      }
    }
    __syncthreads();
    VT bo[P::PARTS][4], ao[P::PARTS][4];
#pragma unroll
    for (int q = 0; q < P::PARTS; ++q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) bo[q][i] = ld8<VT>(&S[q][(TILE + m_off + 16 * i + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int j = 0; j < 4; ++j) ao[q][j] = ld8<VT>(&S[q][(a_off + 16 * j + l % 16) * LDK + 8 * (l / 16)]);
    }
#pragma unroll
    for (int pr = 0; pr < P::NPROD; ++pr) {
      const int pa = kPA[pr], pb = kPB[pr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (P::has_scaled && pr > 0) acc2[i][j] = P::mma(bo[pa][i], ao[pb][j], acc2[i][j]);
          else acc[i][j] = P::mma(bo[pa][i], ao[pb][j], acc[i][j]);
        }
    }
    // empty the FP32 accumulators into FP64 after every stage
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = (double)acc[i][j][r];
          if constexpr (P::has_scaled) v += (double)acc2[i][j][r] * (double)kLoScale;
          wide[i][j][r] += v;
        }
        acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (P::has_scaled) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
      }
  }
  double* Pp = partial + (int64_t)blockIdx.x * a * m;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mi = m0 + m_off + 16 * i + 4 * (l / 16) + r;
        const int ai = a0 + a_off + 16 * j + l % 16;
        if (mi < m && ai < a) Pp[ai + (int64_t)mi * a] = wide[i][j][r];
      }
}

// ---------------------------------------------------------------- nn
// A-side stage: hi/lo[row][k] (8 k per 16-byte group); B-side: [col][k].
template <int MATH, int MODE>
__global__ __launch_bounds__(NT) void nn_lowp_kernel(NnArgs p) {
  typedef Lp<MATH> P;
  typedef typename P::e_t E;
  typedef typename P::v_t VT;
  __shared__ __attribute__((aligned(16))) E As[P::PARTS][TILE * LDK];
  __shared__ __attribute__((aligned(16))) E Bs[P::PARTS][TILE * LDK];
  __shared__ double mean[TILE];
  int64_t rt;
  int ct;
  xcd_tile_map(blockIdx.x, p.n_row_tiles, p.n_col_tiles, &rt, &ct);
  if (rt >= p.n_row_tiles) return;
  const int64_t row0 = rt * TILE;
  const int col0 = ct * TILE;
  const float* __restrict__ A = static_cast<const float*>(p.A);
  const int t = threadIdx.x, l = t % kWave, w = t / kWave;
  const int c_off = (w / 2) * 64, r_off = (w % 2) * 64;
  if constexpr (MODE == NN_ANALYSIS) {
    __shared__ double part[2][TILE];
    const int rr = t % TILE, q = t / TILE;
    const int64_t row = row0 + rr;
    double s = 0.0;
    if (row < p.n)
      for (int j = q; j < p.K; j += 2) s += (double)A[row + (int64_t)j * p.lda];
    part[q][rr] = s;
    __syncthreads();
    if (t < TILE) mean[t] = (part[0][t] + part[1][t]) / (double)p.K;
    __syncthreads();
  }
  mf_f4 acc[4][4], acc2[P::has_scaled ? 4 : 1][P::has_scaled ? 4 : 1];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (P::has_scaled) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc2[i][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int k0 = 0; k0 < p.K; k0 += KC) {
    // A-side items: (row, 8-k group): TILE rows x KC/8 groups = 512 items
    float av[2][8];
    double bv[2][8];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int item = it * NT + t;
      const int rr = item % TILE, kg = item / TILE;
      const int64_t row = row0 + rr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * kg + e;
        float v = 0.f;
        if (row < p.n && k < p.K) {
          v = A[row + (int64_t)k * p.lda];
          if constexpr (MODE == NN_ANALYSIS) v = (float)((double)v - mean[rr]);
        }
        av[it][e] = v;
      }
      // B-side items: (col, 8-k group): TILE cols x KC/8 groups
      const int cc = item % TILE;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * kg + e;
        bv[it][e] = (k < p.K && col0 + cc < p.m) ? p.scale * p.Bm[k + (int64_t)(col0 + cc) * p.ldb] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int item = it * NT + t;
      const int rr = item % TILE, kg = item / TILE;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        E pa[P::PARTS], pb[P::PARTS];
        P::conv(av[it][e], pa);
        P::conv((float)bv[it][e], pb);
#pragma unroll
        for (int q = 0; q < P::PARTS; ++q) {
          As[q][rr * LDK + 8 * kg + e] = pa[q];
          Bs[q][rr * LDK + 8 * kg + e] = pb[q];
        }
      }
    }
    __syncthreads();
    VT co[P::PARTS][4], ro[P::PARTS][4];
#pragma unroll
    for (int q = 0; q < P::PARTS; ++q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) co[q][i] = ld8<VT>(&Bs[q][(c_off + 16 * i + l % 16) * LDK + 8 * (l / 16)]);
#pragma unroll
      for (int j = 0; j < 4; ++j) ro[q][j] = ld8<VT>(&As[q][(r_off + 16 * j + l % 16) * LDK + 8 * (l / 16)]);
    }
#pragma unroll
    for (int pr = 0; pr < P::NPROD; ++pr) {
      const int pa = kPA[pr], pb = kPB[pr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (P::has_scaled && pr > 0) acc2[i][j] = P::mma(co[pa][i], ro[pb][j], acc2[i][j]);
          else acc[i][j] = P::mma(co[pa][i], ro[pb][j], acc[i][j]);
        }
    }
  }
  float* __restrict__ Cout = static_cast<float*>(p.Cout);
  const float* __restrict__ Cin = static_cast<const float*>(p.Cin);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + c_off + 16 * i + 4 * (l / 16) + r;
        const int64_t row = row0 + r_off + 16 * j + l % 16;
        if (col < p.m && row < p.n) {
          double prod = (double)acc[i][j][r];
          if constexpr (P::has_scaled) prod += (double)acc2[i][j][r] * (double)kLoScale;
          const double cin = (double)Cin[row + (int64_t)col * p.ldc];
          const double out = (MODE == NN_UPDATE) ? cin - prod : cin + prod;
          Cout[row + (int64_t)col * p.ldo] = (float)out;
        }
      }
}

template <int MATH>
void tn_launch(dim3 grid, hipStream_t s, int64_t n, int a, int m, const float* A, int64_t lda, const float* B,
               int64_t ldb, double* partial, int64_t rpc, int tiles_m, bool vec) {
  tn_lowp_kernel<MATH><<<grid, NT, 0, s>>>(n, a, m, A, lda, B, ldb, partial, rpc, tiles_m, vec);
}

template <int MATH>
void nn_launch(unsigned g, hipStream_t s, int mode, const NnArgs& p) {
  if (mode == NN_ANALYSIS) nn_lowp_kernel<MATH, NN_ANALYSIS><<<g, NT, 0, s>>>(p);
  else nn_lowp_kernel<MATH, NN_UPDATE><<<g, NT, 0, s>>>(p);
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
  const int tiles = ((a + TILE - 1) / TILE) * tiles_m;
  if (tiles > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "tn product: too many output tiles");
  const bool vec = ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0 && (lda % 4) == 0 && (ldb % 4) == 0;
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
  p.n_row_tiles = (p.n + TILE - 1) / TILE;
  p.n_col_tiles = (p.m + TILE - 1) / TILE;
  const int64_t groups = (p.n_row_tiles + 7) / 8;
  const int64_t blocks = groups * 8 * p.n_col_tiles;
  if (blocks > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "nn product: grid too large");
  const unsigned g = (unsigned)blocks;
  switch (math) {
    case ENKF_MATH_BF16: nn_launch<ENKF_MATH_BF16>(g, s, mode, p); break;
    case ENKF_MATH_F16: nn_launch<ENKF_MATH_F16>(g, s, mode, p); break;
    case ENKF_MATH_BF16X3: nn_launch<ENKF_MATH_BF16X3>(g, s, mode, p); break;
    case ENKF_MATH_F16X2: nn_launch<ENKF_MATH_F16X2>(g, s, mode, p); break;
    default: return fail(ENKF_ERR_INVALID_ARG, "nn product: not a narrow math type");
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
