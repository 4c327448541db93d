// Launchers of the blocked-solve helper kernels (panel_kernels.hip).
#pragma once

#include "enkf_internal.h"

namespace enkf {

constexpr int kMaxPanel = 128;   // panel widths up to 128 (two packed b x b triangles fit in LDS)

// Y = R^{-1} X row by row (Step 1); latches NOT_SPD for r_i <= 0 or non-finite.
enkf_status launch_scale_rows(enkf_dtype dt, int64_t n, int m, const void* X, int64_t ldx, const double* r, void* Y,
                              int64_t ldy, unsigned* status, hipStream_t s);
// M = I + sym(P[:, :b]) = L D L^T (L unit lower); gamma_out[0..b) = D;
// S = D^{-1/2} L^{-1} (b x b lower triangular, ld b), so M^{-1} = S^T S.
enkf_status launch_panel_factor(int b, const double* P, int64_t ldp, double* gamma_out, double* S, unsigned* status,
                                hipStream_t s);
// Q (b x m, ld b) = M^{-1} Pr = S^T (S Pr), Pr b x m with leading dimension ldp.
enkf_status launch_panel_apply(int b, int m, const double* S, const double* Pr, int64_t ldp, double* Q,
                               hipStream_t s);

// FP64 -> FP32 copy divided by the rms of X (sumsq: device ||X||_F^2, or
// NULL for no scaling) and, with r, by r_i row by row (Step 1 fused; bad r_i
// latch NOT_SPD in status). The way back to FP64 is the last panel update of
// each solve, which multiplies by the same rms.
enkf_status launch_convert(int64_t n, int m, const double* X, int64_t ldx, float* Y, int64_t ldy, const double* sumsq,
                           const double* r, unsigned* status, hipStream_t s);
// Z += X, FP64.
enkf_status launch_add(int64_t n, int m, const double* X, int64_t ldx, double* Z, int64_t ldz, hipStream_t s);
// out[0] = ||X||_F^2, or ||R^{-1} X||_F^2 when r is given (fixed-order
// two-stage sum; part holds norm_partial_elems() doubles).
int norm_partial_elems();
enkf_status launch_sumsq(int64_t n, int m, const double* X, int64_t ldx, const double* r, double* part, double* out,
                         hipStream_t s);

}  // namespace enkf
