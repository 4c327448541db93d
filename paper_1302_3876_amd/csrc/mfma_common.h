// Matrix-core (MFMA) building blocks for gfx950, wave64.
//
// Shapes used: 16x16x4 in FP64 and FP32 (one A and one B element per lane),
// 16x16x32 in BF16 and FP16 with FP32 accumulation (eight of each per lane).
// Operand layouts (lane l, 0..63):
//   16x16x4 : A[i][k] with i = l%16, k = l/16;     B[k][j] with k = l/16, j = l%16
//   16x16x32: A[i][k] with i = l%16, k = 8(l/16)+e; B[k][j] with k = 8(l/16)+e, j = l%16
// Result (16x16, four values per lane, register r):
//   FP32 accumulators: row 4(l/16)+r, column l%16
//   FP64 accumulators: row l/16+4r,   column l%16
#pragma once

#include <hip/hip_runtime.h>

namespace enkf {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));

struct MfmaF64 {
  typedef mf_d4 acc_t;
  typedef double op_t;
  static constexpr int KSTEP = 4;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return l / 16 + 4 * r; }
};

struct MfmaF32 {
  typedef mf_f4 acc_t;
  typedef float op_t;
  static constexpr int KSTEP = 4;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l / 16) + r; }
};

struct MfmaBF16 {
  typedef mf_f4 acc_t;
  typedef mf_bf8 op_t;
  static constexpr int KSTEP = 32;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l / 16) + r; }
};

struct MfmaF16 {
  typedef mf_f4 acc_t;
  typedef mf_h8 op_t;
  static constexpr int KSTEP = 32;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(op_t a, op_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l / 16) + r; }
};

// Map a 1-D block index to (row tile, column tile) so that the column tiles
// of one row tile run back to back on the same XCD (blocks are dealt to the
// 8 XCDs round-robin): the row tile's operand stays in that XCD's L2.
__device__ __forceinline__ void xcd_tile_map(int64_t bid, int64_t n_row_tiles, int n_col_tiles, int64_t* rt,
                                             int* ct) {
  const int64_t xcd = bid % 8, local = bid / 8;
  const int64_t group = local / n_col_tiles;
  *ct = (int)(local % n_col_tiles);
  *rt = group * 8 + xcd;
  (void)n_row_tiles;
}

}  // namespace enkf
