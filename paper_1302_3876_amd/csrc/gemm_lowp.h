// Launchers of the narrow-input (BF16/F16 and their split forms) products.
#pragma once

#include "enkf_internal.h"
#include "gemm_mfma.h"

namespace enkf {

// G (a x m, FP64) = A^T B with FP32 operands rounded to `math` in LDS.
enkf_status launch_tn_lowp(enkf_math math, int64_t n, int a, int m, const float* A, int64_t lda, const float* B,
                           int64_t ldb, double* G, int64_t ldg, double* partial, hipStream_t s);
// NN_UPDATE or NN_ANALYSIS with FP32 storage and `math` inputs.
enkf_status launch_nn_lowp(enkf_math math, int mode, NnArgs p, hipStream_t s);

}  // namespace enkf
