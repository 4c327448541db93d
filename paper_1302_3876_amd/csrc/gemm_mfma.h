// Launchers of the matrix-core products (gemm_mfma.hip).
#pragma once

#include "enkf_internal.h"

namespace enkf {

// NN_UPDATE64 (FP32 storage; FP32 or narrow inputs): the updated X goes to
// Z64 in FP64 (Z64 = s (X - A B), or Z64 += s (X - A B) with z64_acc; s the
// rms scale of the FP16 forms, else 1) instead of back to Cout.
enum NnMode : int { NN_UPDATE = 0, NN_ANALYSIS = 1, NN_RESIDUAL = 2, NN_UPDATE64 = 3 };

struct NnArgs {
  int64_t n;            // rows
  int K;                // inner dimension (columns of A, rows of Bm)
  int m;                // output columns
  const void* A; int64_t lda;        // n x K, storage type
  const double* Bm; int64_t ldb;     // K x m, FP64
  double scale;                      // Bm is multiplied by scale (ANALYSIS); 1 otherwise
  const void* Cin; int64_t ldc;      // UPDATE: X; ANALYSIS: XB; RESIDUAL: Z
  void* Cout; int64_t ldo;           // UPDATE: X (same as Cin); ANALYSIS: XA; RESIDUAL: rho
  float* Cout32; int64_t ldo32;      // RESIDUAL, optional: R^{-1} rho in FP32 here instead of rho in Cout
  const void* Din; int64_t ldd;      // RESIDUAL: D
  const double* r;                   // RESIDUAL: diag(R)
  void* bws;                         // workspace: Bm converted (nn_bt_bytes(K, m) bytes)
  double* part; int64_t part_cap;    // RESIDUAL, optional: per-block sums of rho^2 (capacity in doubles)
  double* sumsq;                     // RESIDUAL with part: ||rho||_F^2, the partials summed in a fixed order
  double* Z64; int64_t ldz64;        // UPDATE64: FP64 destination of the updated X
  int z64_acc;                       // UPDATE64: 1 adds to Z64, 0 overwrites it
  const double* z64_sumsq;           // UPDATE64, optional: the result is multiplied by rms_scale(z64_sumsq, n m)
  int64_t n_row_tiles;               // set by the launcher
  int n_col_tiles;                   // set by the launcher
};

// G (a x m, FP64, ldg) = A^T B with split-K partials (partial must hold
// tn_partial_elems doubles); matrix cores in the storage precision.
int64_t tn_partial_elems(int64_t n, int a, int m);
enkf_status launch_tn(enkf_dtype dt, int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb,
                      double* G, int64_t ldg, double* partial, hipStream_t s);

enkf_status launch_nn(enkf_dtype dt, int mode, NnArgs p, hipStream_t s);
// Capacity (doubles) of NnArgs::part that any RESIDUAL product with n rows
// and at most m columns needs.
int64_t nn_residual_part_elems(int64_t n, int m);
// Converted right factor of an nn product: padded rows (multiple of 32),
// padded columns (multiple of 128), workspace bytes.
int nn_bt_rows(int K);
int nn_bt_cols(int m);
size_t nn_bt_bytes(int K, int m);
// G (a x m, ldg) = sum over `chunks` partials of a x m (fixed order).
enkf_status launch_partial_sum(int a, int m, int64_t chunks, const double* partial, double* G, int64_t ldg,
                               hipStream_t s);

}  // namespace enkf
