// Plain iterative Sherman-Morrison sweeps (Section 3.1, Steps 1-2), one
// kernel launch per level, for gfx950.
//
// A launch updates m active columns x_q of X (the U columns k+1..N during
// the factorisation, every Z column during a solve, or both at once when
// the factorisation and a solve run together, as in the level loop of
// Section 3.3):
//     Step 1 (eq. SM-step-1):  x_q = src_q / r
//     level k (eq. SM-step-2): x_q <- x_q - h_k c_q,  h_k = u_k^{(k-1)} / gamma_k,
//                              c_q = v_k^T x_q  (reduced by the previous launch)
// and, fused into the same pass, the products of the NEXT level,
//     c'_q = v_{k+1}^T x_q(new),
// so each level reads and writes its active columns exactly once. Each block
// leaves one partial of c'_q per column (shuffles within a wave, then LDS
// across waves). Every block of the next launch sums, by itself and in the
// same fixed order, the partials of the columns it updates: no atomics or
// cross-block fences (which on a multi-XCD part would write back the L2), and
// results are bitwise reproducible. During the factorisation the products of
// the pivot column give gamma_k = 1 + v_k^T u_k^{(k-1)}; block (0,0) stores it
// and latches a status error if it is not finite or not > 0 (Section 3.3).
//
// Layout: column-major, threads own consecutive row chunks of VW elements
// (16-byte loads), a block owns COLS columns of one tile of LV_THREADS*VW*RPT
// rows or, past lv_max_row_blocks tiles, of several consecutive tiles (the
// partials it sums and leaves are per block, so their number stays bounded).
#include "enkf_internal.h"

namespace enkf {
namespace {

constexpr int LV_THREADS = 256;
constexpr int LV_WAVES = LV_THREADS / kWave;
constexpr int LV_COLS = 8;
constexpr int LV_RPT = 2;
// Streamed launches (columns past the last-level cache): a quarter of the
// columns per block and four times the rows, so fewer column streams are
// open at once. Narrow groups re-read u_k and v_{k+1} once per group; with
// the chunked grid order below those re-reads hit the L2. n = 2^21, 512 down
// to 256 columns per level, level time per solve with chunks of 256: 2 x 8
// 556-558 ms, 4 x 4 591-592, 4 x 8 598, 8 x 2 629 (unchunked: 2 x 8 655,
// 4 x 4 603-625, 8 x 2 636, 16 x 2 646).
constexpr int LV_COLS_STREAM = 2;
constexpr int LV_RPT_STREAM = 8;
template <bool STREAM> constexpr int lv_cols() { return STREAM ? LV_COLS_STREAM : LV_COLS; }
template <bool STREAM> constexpr int lv_rpt() { return STREAM ? LV_RPT_STREAM : LV_RPT; }
// Row blocks of a launch at most: 256, and 512 from 2048 tiles up (n >= 2^21
// FP64 rows). c3 (n = 2^21, N = 256) factor + solve: 624 ms with 256 (each
// block walking 4 tiles), 606 with 512 and 640, 614 with 768, 621 with 1024,
// 625 with 384; n = 2^20, N = 96: 41.1 ms with 256, 41.7 with 512. A function
// of n alone, so that every launch of a sweep has the same partial layout.
inline int64_t lv_max_row_blocks(int64_t tiles) { return tiles >= 2048 ? 512 : 256; }
// Streamed launches run their row blocks in chunks of LV_CHUNK_STREAM: every
// column group of one chunk before the next chunk (a bijection of the grid
// onto (row block, column group); a row block keeps its XCD, as the chunk is
// a multiple of 8). With 512 row blocks and 4 x 4 groups, c3 level time per
// solve: 603 ms unchunked, 592 with chunks of 256, 622 of 128, 658 of 64;
// with 768 row blocks 611 (chunks of 256 or 384), with 1024 599 (512) and
// 705 (256). With 2 x 8 groups: 556-558 ms (256), 556 (128).
constexpr int LV_CHUNK_STREAM = 256;

template <typename T, int VW> struct VecT;
template <> struct VecT<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecT<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct VecT<double, 1> { typedef double type; };
template <> struct VecT<float, 1> { typedef float type; };

// Loads and stores of VW consecutive rows. The launcher picks VW > 1 only
// when columns are 16-byte aligned and VW divides n, so a vector is wholly
// inside or wholly outside the rows; callers pass a valid row index (rows
// past n are redirected to row 0 and their values never stored), so loads
// carry no branches and all of a block's loads are in flight together.
// STREAM: non-temporal accesses, for columns that are read and written once
// per level and whose level working set exceeds the last-level cache (they
// would only evict the vectors every column group re-reads).
template <typename T, int VW, bool STREAM = false>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, int64_t row, T (&v)[VW]) {
  typedef typename VecT<T, VW>::type vt;
  vt x;
  if constexpr (STREAM) x = __builtin_nontemporal_load(reinterpret_cast<const vt*>(p + row));
  else x = *reinterpret_cast<const vt*>(p + row);
  if constexpr (VW == 1) {
    v[0] = x;
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) v[e] = x[e];
  }
}

template <typename T, int VW, bool STREAM = false>
__device__ __forceinline__ void store_vec(T* __restrict__ p, int64_t row, const T (&v)[VW]) {
  typedef typename VecT<T, VW>::type vt;
  vt x;
  if constexpr (VW == 1) {
    x = v[0];
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) x[e] = v[e];
  }
  if constexpr (STREAM) __builtin_nontemporal_store(x, reinterpret_cast<vt*>(p + row));
  else *reinterpret_cast<vt*>(p + row) = x;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Lane-strided sum of nb partials: lane l adds p[l], p[l+64], ... in that
// order (loads issued four at a time).
__device__ __forceinline__ double lane_strided_sum(const double* __restrict__ p, int nb, int lane) {
  double s = 0.0;
  int b = lane;
  for (; b + 3 * kWave < nb; b += 4 * kWave) {
    const double x0 = p[b], x1 = p[b + kWave], x2 = p[b + 2 * kWave], x3 = p[b + 3 * kWave];
    s += x0;
    s += x1;
    s += x2;
    s += x3;
  }
  for (; b < nb; b += kWave) s += p[b];
  return s;
}

// Sum of one value per thread over the block, returned to every thread, in a
// fixed order (shuffle tree per wave, then waves 0..3).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < LV_WAVES; ++w) s += red[w];
  return s;
}

// MULTI: the grid has fewer row blocks than tiles and a block walks its
// consecutive tiles (a separate instance: one-tile launches keep their
// register budget).
template <typename T, int VW, bool STEP1, bool LOOKAHEAD, bool OWN_GAMMA, bool MULTI, bool STREAM>
__global__ __launch_bounds__(LV_THREADS) void level_kernel(LevelArgs a) {
  constexpr int COLS = lv_cols<STREAM>(), RPT = lv_rpt<STREAM>();
  constexpr int64_t RPB = (int64_t)LV_THREADS * VW * RPT;   // rows of one tile
  const int64_t n = a.n;
  const int nb = gridDim.x;
  int bx = blockIdx.x, by = blockIdx.y;            // row block, column group
  if constexpr (STREAM) {
    if (nb % LV_CHUNK_STREAM == 0) {
      const int64_t lin = (int64_t)blockIdx.y * nb + blockIdx.x;   // dispatch order
      const int64_t per = (int64_t)LV_CHUNK_STREAM * gridDim.y;
      const int64_t chunk = lin / per, rem = lin % per;
      by = (int)(rem / LV_CHUNK_STREAM);
      bx = (int)(chunk * LV_CHUNK_STREAM + rem % LV_CHUNK_STREAM);
    }
  }
  int64_t tile0 = bx, tile1 = tile0 + 1;
  if constexpr (MULTI) {
    const int64_t tiles = (n + RPB - 1) / RPB;
    const int64_t tpb = (tiles + nb - 1) / nb;
    tile0 = (int64_t)bx * tpb;
    tile1 = min(tiles, tile0 + tpb);
  }
  const int g = by;
  const int col0 = g * COLS;
  const int ncol = min(COLS, a.m - col0);
  const int t = threadIdx.x;
  const int lane = t % kWave, wave = t / kWave;
  T* __restrict__ X = static_cast<T*>(a.X);
  T* __restrict__ Out = a.dst ? static_cast<T*>(a.dst) : X;
  const int64_t ldo = a.dst ? a.ldo : a.ldx;
  const int32_t* __restrict__ cmap = a.colmap;
  // column (of X, and partial slot) of active column q
  auto phys = [&](int q) -> int { return cmap ? cmap[q] : q; };
  const T* __restrict__ ukp = static_cast<const T*>(a.uk);
  if (!STEP1 && a.uk_idx) ukp += (int64_t)(*a.uk_idx) * a.ldu_idx;
  const T* __restrict__ vnp = static_cast<const T*>(a.vnext);
  if (LOOKAHEAD && a.vn_idx) vnp += (int64_t)(*a.vn_idx) * a.ldv_idx;
  const T* __restrict__ src = STEP1 ? static_cast<const T*>(a.src) : X;
  const int64_t lds = STEP1 ? a.lds : a.ldx;

  int64_t rows[RPT], rowc[RPT];
  T xv[COLS][RPT][VW];
  T uv[RPT][VW], vv[RPT][VW];
  // 1. Every load of a tile at once: the active columns (a column past the
  //    last reads the last one and is not stored; the source of Step 1 may
  //    be the destination itself), u_k and v_{k+1}.
  auto load_tile = [&](int64_t tile) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      rows[r] = tile * RPB + ((int64_t)r * LV_THREADS + t) * VW;
      rowc[r] = rows[r] < n ? rows[r] : 0;
    }
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      const T* __restrict__ col = src + (int64_t)phys(min(col0 + c, a.m - 1)) * lds;
#pragma unroll
      for (int r = 0; r < RPT; ++r) load_vec<T, VW, STREAM>(col, rowc[r], xv[c][r]);
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      if constexpr (!STEP1) load_vec<T, VW>(ukp, rowc[r], uv[r]);
      if constexpr (LOOKAHEAD) load_vec<T, VW>(vnp, rowc[r], vv[r]);
    }
  };
  load_tile(tile0);
  __builtin_amdgcn_sched_barrier(0);

  // 2. Products c_q = v_k^T x_q of this block's columns (and of the pivot
  //    column when forming gamma_k), from the previous launch's partials,
  //    once per block while the first tile's loads are in flight.
  __shared__ double cq_s[COLS];
  __shared__ double gam_s;
  if constexpr (!STEP1) {
    const int nred = ncol + (OWN_GAMMA ? 1 : 0);
    for (int c = wave; c < nred; c += LV_WAVES) {
      const int pc = (c < ncol) ? (cmap ? cmap[col0 + c] : col0 + c + a.prev_off) : 0;
      double sacc = lane_strided_sum(a.prev + (int64_t)pc * nb, nb, lane);
      sacc = wave_sum(sacc);
      if (lane == 0) {
        if (c < ncol) cq_s[c] = sacc;
        else gam_s = sacc;
      }
    }
    __syncthreads();
  }
  double inv_gamma = 0.0;
  if constexpr (!STEP1) {
    double gam;
    if constexpr (OWN_GAMMA) {
      gam = 1.0 + gam_s;
      if (bx == 0 && by == 0 && t == 0) {
        *a.gamma_out = gam;
        if (!(gam > 0.0) || !__builtin_isfinite(gam)) atomicOr(a.status, kStatusNotSpd);
      }
    } else {
      gam = *a.gamma_in;
    }
    inv_gamma = 1.0 / gam;
  }
  double acc[COLS];
#pragma unroll
  for (int c = 0; c < COLS; ++c) acc[c] = 0.0;
  for (int64_t tile = tile0; tile < tile1; ++tile) {
    if (tile != tile0) load_tile(tile);
    // 3. Per-row factors: 1/r_i (Step 1) or h_k[i] = u_k[i] / gamma_k (level).
    double hrow[RPT][VW];
    double vn[RPT][VW];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const bool ok = rows[r] < n;
      if constexpr (STEP1) {
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const double rv = a.r ? a.r[rowc[r] + e] : 1.0;   // no r: Step 1 already applied (block R)
          if (ok && (!(rv > 0.0) || !__builtin_isfinite(rv))) atomicOr(a.status, kStatusNotSpd);
          hrow[r][e] = ok ? 1.0 / rv : 0.0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) hrow[r][e] = ok ? (double)uv[r][e] * inv_gamma : 0.0;
      }
      if constexpr (LOOKAHEAD) {
#pragma unroll
        for (int e = 0; e < VW; ++e) vn[r][e] = ok ? (double)vv[r][e] : 0.0;
      }
    }

    // 4. Update, look-ahead products, stores.
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      double cq = 0.0;
      if constexpr (!STEP1) cq = (c < ncol) ? cq_s[c] : 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          double x = (double)xv[c][r][e];
          x = STEP1 ? x * hrow[r][e] : x - hrow[r][e] * cq;
          xv[c][r][e] = (T)x;
          if constexpr (LOOKAHEAD) acc[c] += vn[r][e] * (double)xv[c][r][e];
        }
        if (c < ncol && rows[r] < n) store_vec<T, VW, STREAM>(Out + (int64_t)phys(col0 + c) * ldo, rows[r], xv[c][r]);
      }
    }
  }
  if constexpr (!LOOKAHEAD) return;

  // One partial per column for this block.
  __shared__ double red[LV_WAVES][COLS];
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (t < ncol) {
    double sacc = 0.0;
#pragma unroll
    for (int w = 0; w < LV_WAVES; ++w) sacc += red[w][t];
    a.part_out[(int64_t)phys(col0 + t) * nb + bx] = sacc;
  }
}

// gamma = 1 + (sum of one partial column), summed exactly as the level
// kernels sum it (lane-strided, then the shuffle tree).
__global__ __launch_bounds__(kWave) void gamma_kernel(const double* __restrict__ part, int nb, int col,
                                                      double* __restrict__ gamma_out, unsigned* status) {
  double sacc = lane_strided_sum(part + (int64_t)col * nb, nb, threadIdx.x);
  sacc = wave_sum(sacc);
  if (threadIdx.x == 0) {
    const double gam = 1.0 + sacc;
    *gamma_out = gam;
    if (!(gam > 0.0) || !__builtin_isfinite(gam)) atomicOr(status, kStatusNotSpd);
  }
}

template <typename T, int VW, bool MULTI, bool STREAM>
enkf_status launch_flags(const LevelArgs& a, dim3 grid, hipStream_t s) {
  const bool step1 = a.src != nullptr, look = a.vnext != nullptr, own = a.gamma_out != nullptr;
  if (step1) {
    if (look) level_kernel<T, VW, true, true, false, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
    else level_kernel<T, VW, true, false, false, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
  } else if (own) {
    if (look) level_kernel<T, VW, false, true, true, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
    else level_kernel<T, VW, false, false, true, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
  } else {
    if (look) level_kernel<T, VW, false, true, false, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
    else level_kernel<T, VW, false, false, false, MULTI, STREAM><<<grid, LV_THREADS, 0, s>>>(a);
  }
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

// Last-level (infinity) cache of the MI355X: 256 MiB. A launch whose active
// columns exceed it streams them with non-temporal accesses.
constexpr double kLvMallBytes = 256.0 * 1024.0 * 1024.0;

template <typename T, int VW>
enkf_status launch_t(const LevelArgs& a, hipStream_t s) {
  if (a.m <= 0) return ENKF_SUCCESS;
  const int64_t nb = level_row_blocks(ENKF_F64, VW, a.n);
  const bool stream = (double)a.m * (double)a.n * sizeof(T) > kLvMallBytes;
  const int cols = stream ? lv_cols<true>() : lv_cols<false>();
  const int ng = (a.m + cols - 1) / cols;
  if (nb > 0x7fffffff || ng > 65535) return fail(ENKF_ERR_NOT_SUPPORTED, "level sweep: problem too large for grid");
  const int64_t rpb = (int64_t)LV_THREADS * VW * (stream ? lv_rpt<true>() : lv_rpt<false>());
  const dim3 grid((unsigned)nb, (unsigned)ng);
  if (nb < (a.n + rpb - 1) / rpb)
    return stream ? launch_flags<T, VW, true, true>(a, grid, s) : launch_flags<T, VW, true, false>(a, grid, s);
  return stream ? launch_flags<T, VW, false, true>(a, grid, s) : launch_flags<T, VW, false, false>(a, grid, s);
}

}  // namespace

int level_vw(enkf_dtype dt) { return dt == ENKF_F64 ? 2 : 4; }

// Row blocks of a level launch: one tile of LV_THREADS*VW*LV_RPT rows each,
// up to lv_max_row_blocks; past that a block walks several consecutive tiles,
// so the previous launch's partials that every block sums stay few.
int level_row_blocks(enkf_dtype, int vw, int64_t n) {
  const int64_t rpb = (int64_t)LV_THREADS * vw * LV_RPT;
  const int64_t tiles = (n + rpb - 1) / rpb;
  const int64_t cap = lv_max_row_blocks(tiles);
  const int64_t tpb = (tiles + cap - 1) / cap;
  return (int)((tiles + tpb - 1) / tpb);
}

enkf_status launch_level(enkf_dtype dt, const LevelArgs& a, hipStream_t s) {
  if (dt == ENKF_F64) return a.vw == 2 ? launch_t<double, 2>(a, s) : launch_t<double, 1>(a, s);
  return a.vw == 4 ? launch_t<float, 4>(a, s) : launch_t<float, 1>(a, s);
}

enkf_status launch_gamma_from_partials(const double* part, int nb, int col, double* gamma_out, unsigned* status,
                                       hipStream_t s) {
  gamma_kernel<<<1, kWave, 0, s>>>(part, nb, col, gamma_out, status);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

}  // namespace enkf
