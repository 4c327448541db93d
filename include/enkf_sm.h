/*
 * enkf_sm.h -- C ABI of the MI355X (gfx950) EnKF analysis library.
 *
 * The library computes the analysis step of the ensemble Kalman filter with
 * the iterative Sherman-Morrison formula of Nino-Ruiz, Sandu and Anderson,
 * "An efficient implementation of the ensemble Kalman filter based on an
 * iterative Sherman-Morrison formula" (Statistics and Computing, 2014):
 *
 *   D  = Y - H X^B,  V = H S,  S = (X^B - xbar 1^T) / sqrt(N-1)    (Section 3, eq. system-rewritten)
 *   Z  = S*(R, V, D), i.e. (R + V V^T) Z = D, R diagonal          (Section 3.1, Steps 1-2)
 *   X^A = X^B + S (V^T Z)                                         (Section 3.1, the SMEnKF listing)
 *
 * Conventions for every call:
 *   - Matrices are column-major, one column per ensemble member: element
 *     (i, j) of a matrix with leading dimension ld sits at p[i + j*ld].
 *   - Every data pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's data_ptr) unless the argument says HOST.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Every call only enqueues work on that stream and returns; nothing is
 *     synchronised unless the argument list says so.
 *   - The caller owns every buffer it passes. A plan borrows the r and V
 *     pointers given to enkf_sm_init (or the last refactor): they must stay
 *     valid and unchanged until enkf_sm_destroy, since the solves, the FP64
 *     refinement residuals and the analysis read them again. (A copy would
 *     double V's footprint: 4 GiB in FP64 at n = 2^21, N = 256.) A plan owns
 *     its workspace (allocated in enkf_sm_init).
 *   - Every call returns an enkf_status. Argument errors are found on the host
 *     before anything is launched. Errors found by kernels (a pivot gamma_k not
 *     finite or not > 0, an r_i not finite or not > 0) are latched in a device
 *     status word of the plan and returned by the next synchronising call
 *     (enkf_sm_solve with info != NULL, or enkf_sm_get_info).
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef ENKF_SM_H
#define ENKF_SM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ENKF_SUCCESS = 0,
    ENKF_ERR_INVALID_ARG = 1,     /* bad shape, leading dimension, pointer or option */
    ENKF_ERR_NOT_SPD = 2,         /* r_i <= 0 / non-finite, or gamma_k <= 0 / non-finite (Section 3.3) */
    ENKF_ERR_NO_CONVERGENCE = 3,  /* refinement stopped above its tolerance; Z holds the last iterate */
    ENKF_ERR_HIP = 4,             /* a HIP runtime call failed */
    ENKF_ERR_OUT_OF_MEMORY = 5,   /* workspace allocation failed */
    ENKF_ERR_NOT_SUPPORTED = 6    /* valid but unsupported combination of options */
} enkf_status;

/* Storage type of V, D, Z, X^B and X^A as the caller passes them. */
typedef enum { ENKF_F64 = 0, ENKF_F32 = 1 } enkf_dtype;

/* ENKF_SM_PLAIN: the level-by-level iteration of Section 3.1 (Step 2), one
 *   pass over the active columns per level k = 1..N.
 * ENKF_SM_BLOCKED: the same levels taken b at a time. A panel K of b levels
 *   applies the Sherman-Morrison-Woodbury identity (eq. SWM) with a rank-b
 *   term: X <- X - U_K M_K^{-1} (V_K^T X), M_K = I + V_K^T U_K, whose LDL^T
 *   pivots are exactly the gamma_k of the b levels. */
typedef enum { ENKF_SM_PLAIN = 0, ENKF_SM_BLOCKED = 1 } enkf_sm_algo;

/* Input type of the blocked panel products V^T U, V^T X and U Q on the matrix
 * cores. A type narrower than `dtype` makes the solve mixed precision: the
 * plan keeps an FP32 copy of V and of the factor, the panel products run in
 * `math`, the b x b panel pivots stay FP64, and enkf_sm_solve refines Z with
 * FP64 residuals D - (R Z + V (V^T Z)). The split forms carry more of each
 * FP32 operand: BF16X3 writes it as the sum of three BF16 parts (8 bits of
 * significand each) and sums the six cross products of significance at
 * least 2^-16 relative to the leading one; F16X2 writes it as an FP16 high
 * part plus an FP16 low part stored scaled by 2^11 (11 bits each) and sums
 * three cross products. Accumulation is FP32 in every form. */
typedef enum {
    ENKF_MATH_F64 = 0,
    ENKF_MATH_F32 = 1,
    ENKF_MATH_BF16 = 2,
    ENKF_MATH_F16 = 3,
    ENKF_MATH_BF16X3 = 4,
    ENKF_MATH_F16X2 = 5
} enkf_math;

/* Pivoting of Section 3.4 (eq. gamma-value): before level k the remaining
 * column with the largest gamma is swapped into position k. Plain only. */
#define ENKF_FLAG_PIVOT 0x1u
/* Diagnostics (FP64 storage, diagonal R, n_ens <= 4096; ignored otherwise):
 * every synchronous solve (info != NULL) reports the relative residual and
 * the normwise backward error of its Z,
 *   eta = ||D - W Z||_F / (||W||_2 ||Z||_F + ||D||_F),
 * with ||W||_2 estimated per factorisation as max r + the Rayleigh quotient
 * of V^T V after 60 power steps (at most 2 ||W||_2; the N x N Gram costs
 * 2 n N^2 flops). Plain and unrefined blocked solves form one FP64
 * residual D - (R Z + V (V^T Z)) for it; an in-place solve (Z overwrote D)
 * reports -1. */
#define ENKF_FLAG_DIAGNOSE 0x2u
/* Panel width by measurement (BLOCKED with block = 0): enkf_sm_init times
 * the factorisation and one solve of min(N, max_nrhs) right-hand sides (the
 * columns of V; no refinement) on the plan's own data for b = 32, 64, 96,
 * 128 (those <= N) and keeps the fastest (eq. SWM with a rank-b term: the
 * panel products grow with b, the passes over the trailing columns shrink
 * as 1/b). A shape (n_obs, n_ens, dtype, math, max_nrhs) tuned before in
 * the process reuses its width. Without the flag, block = 0 is min(N, 128).
 * The timing allocates a scratch right-hand side for the duration of init. */
#define ENKF_FLAG_AUTOTUNE 0x4u

typedef struct {
    int64_t n_obs;          /* n >= 1 */
    int32_t n_ens;          /* N >= 1 */
    enkf_dtype dtype;
    enkf_sm_algo algo;
    enkf_math math;         /* must be ENKF_MATH_F64 for PLAIN F64, ENKF_MATH_F32 for PLAIN F32 */
    int32_t block;          /* panel width b for BLOCKED (1..N); 0 = pick one */
    int32_t max_nrhs;       /* largest nrhs a solve may pass; 0 = n_ens */
    int32_t refine_max_iter;/* blocked: maximum FP64 refinement steps (0 = none). Mixed precision, or
                               FP64 panels (F64/F64): the Woodbury panel update is not backward
                               stable, residual corrections restore FP64 accuracy */
    double refine_tol;      /* refinement: stop when ||D - W Z||_F / ||D||_F <= tol */
    uint32_t flags;         /* ENKF_FLAG_* */
} enkf_sm_desc;

typedef struct {
    int32_t refine_iters;   /* refinement steps taken by the last solve */
    double rel_residual;    /* ||D - W Z||_F / ||D||_F of the last solve (refined or mixed solves, and
                               every solve with ENKF_FLAG_DIAGNOSE), else -1 */
    double backward_error;  /* eta of the last synchronous solve with ENKF_FLAG_DIAGNOSE, else -1 */
    double gamma_min;       /* smallest and largest pivot gamma_k of the factor */
    double gamma_max;
    int32_t device_status;  /* enkf_status latched by kernels (0 = none) */
    int32_t hip_error;      /* hipPeekAtLastError() of the calling thread when the info was taken (0 = none) */
    int32_t block;          /* panel width in use (BLOCKED; 1 for PLAIN) */
} enkf_sm_info;

typedef struct enkf_sm_plan_s* enkf_sm_plan;

/* Host-only check of a descriptor (no GPU needed). */
enkf_status enkf_sm_validate_desc(const enkf_sm_desc* desc);

/*
 * Build the inputs of the solve from the background ensemble (Section 2 and
 * Section 3, eqs. EnSM:Matrix-member-deviations, system-rhs,
 * member-observations), with H the row selection x -> x[obs_idx]:
 *   xbar_s = (1/N) sum_j X^B[s, j]
 *   V[i, j] = (X^B[obs_idx[i], j] - xbar_{obs_idx[i]}) / sqrt(N - 1)
 *   D[i, j] = (y[i] + E[i, j]) - X^B[obs_idx[i], j]
 * XB (n_state x N, ldx >= n_state), obs_idx (n_obs, int64, 0 <= idx < n_state),
 * y (n_obs, FP64), E (n_obs x N, lde >= n_obs, perturbations ~ N(0, R), in
 * `dtype`), V and D (n_obs x N, ldv >= n_obs, in `dtype`). N >= 2.
 * Out-of-range obs_idx entries are not checked on the host (they live on the
 * device); the kernel clamps nothing and the caller must pass valid indices.
 */
enkf_status enkf_build_vd(int64_t n_state, int32_t n_ens, enkf_dtype dtype, const void* XB, int64_t ldx,
                          const int64_t* obs_idx, int64_t n_obs, const double* y, const void* E, int64_t lde,
                          void* V, void* D, int64_t ldv, void* stream);

/*
 * Create a plan and run the D-independent half of S*(R, V, D): Step 1 for V
 * (U0 = R^{-1} V) and the U-updates of every level (eq. SM-step-2-u), which
 * leave the factor {u_k^{(k-1)}, gamma_k} (blocked: {U_K, M_K} per panel).
 * r (n_obs, FP64, each > 0) and V (n_obs x N, ldv >= n_obs, `desc->dtype`)
 * are borrowed until enkf_sm_destroy. Allocates the workspace, so it must not
 * be called under stream capture.
 */
enkf_status enkf_sm_init(enkf_sm_plan* out, const enkf_sm_desc* desc, const double* r, const void* V,
                         int64_t ldv, void* stream);

/*
 * Recompute the factor of an existing plan for a new (r, V) of the same shape
 * and type, reusing its workspace (the next analysis cycle): the same work as
 * enkf_sm_init without any allocation. Clears the latched status word. The
 * new r and V are borrowed as in enkf_sm_init.
 */
enkf_status enkf_sm_refactor(enkf_sm_plan plan, const double* r, const void* V, int64_t ldv);

/*
 * Block-diagonal observation error covariance (Section 2.1: R =
 * diag(R_1, ..., R_B), each R_b SPD of size N_b, sum N_b = n_obs). Step 1
 * (eq. SM-step-1) then applies R^{-1} block by block (Section 3.1; at most
 * O(n N^2) work, Section 3.2) and the level sweeps are unchanged.
 *   offsets: HOST array of n_blocks + 1 row offsets, offsets[0] = 0 <
 *            offsets[1] < ... < offsets[n_blocks] = n_obs, every block of at
 *            most ENKF_MAX_R_BLOCK rows;
 *   blocks:  DEVICE, FP64; block b (rows offsets[b] .. offsets[b+1]-1) is a
 *            dense column-major N_b x N_b matrix stored at
 *            blocks + sum_{c<b} N_c^2. Read at init / refactor only.
 */
#define ENKF_MAX_R_BLOCK 64

typedef struct {
    int64_t n_blocks;
    const int64_t* offsets;
    const double* blocks;
} enkf_block_r;

/*
 * enkf_sm_init with a block-diagonal R. The blocks are factored R_b = L L^T
 * in FP64 on the device (a block that is not SPD latches ENKF_ERR_NOT_SPD),
 * then V as in enkf_sm_init. Plain and blocked algorithms in FP64 or FP32
 * storage; pivoting and the mixed-precision refinement need a diagonal R
 * (ENKF_ERR_NOT_SUPPORTED). Such a plan is refactored with
 * enkf_sm_refactor_block_r (enkf_sm_refactor and enkf_sm_factor_solve return
 * ENKF_ERR_INVALID_ARG) and solved with enkf_sm_solve. Allocates.
 */
enkf_status enkf_sm_init_block_r(enkf_sm_plan* out, const enkf_sm_desc* desc, const enkf_block_r* R, const void* V,
                                 int64_t ldv, void* stream);

/* New block values (same structure) and V: refactor without allocation. */
enkf_status enkf_sm_refactor_block_r(enkf_sm_plan plan, const double* R_blocks, const void* V, int64_t ldv);

/*
 * The D-dependent half of S*: Step 1 for D (Z0 = R^{-1} D) and the Z-updates
 * of every level (eq. SM-step-2-Z): Z = (R + V V^T)^{-1} D.
 * D and Z are n_obs x nrhs (nrhs >= 0; the analysis has nrhs = N) in the
 * plan's dtype. The plain and the unrefined blocked solves may run in place
 * (Z == D with ldz == ldd); refined and mixed-precision solves read D again
 * for every residual and take no overlap of Z and D. Any other overlap is
 * ENKF_ERR_INVALID_ARG. Allocates nothing.
 * info == NULL: asynchronous, refinement (if any) runs exactly
 *   refine_max_iter steps. info != NULL: synchronises the plan's stream,
 *   stops refinement at refine_tol, fills *info and returns latched errors.
 */
enkf_status enkf_sm_solve(enkf_sm_plan plan, int32_t nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz,
                          enkf_sm_info* info);

/*
 * enkf_sm_refactor followed by enkf_sm_solve, as one pass of the level loop
 * of Section 3.3 (Steps 1-2): for the plain algorithm, Step 1 for V and D,
 * then one launch per level k that forms gamma_k (eq. gamma-value) and
 * updates the U columns k+1..N and every Z column together (eq. SM-step-2),
 * so each level reads and writes the active columns of both once. Leaves the
 * same factor as enkf_sm_refactor (later enkf_sm_solve calls reuse it).
 * Arguments and errors as the two calls; the blocked algorithm runs them in
 * sequence. Allocates nothing.
 */
enkf_status enkf_sm_factor_solve(enkf_sm_plan plan, const double* r, const void* V, int64_t ldv, int32_t nrhs,
                                 const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info);

/*
 * Analysis update X^A = X^B + S (V^T Z) with S = (X^B - xbar 1^T)/sqrt(N-1)
 * (Section 3.1), using the plan's V. XB and XA are n_state x N (ldx, ldxa >=
 * n_state) in the plan's dtype; Z is n_obs x N (ldz >= n_obs). XA must not
 * overlap XB (checked on the host). N >= 2. Allocates nothing.
 */
enkf_status enkf_analysis(enkf_sm_plan plan, int64_t n_state, const void* XB, int64_t ldx, const void* Z,
                          int64_t ldz, void* XA, int64_t ldxa);

/*
 * Partially localized analysis update (Section 3.1.2, eq.
 * localized-correction-component):
 *   X^A[i, l] = X^B[i, l] + sum_k S[i, k] sum_j delta(i, j) V[j, k] Z[j, l],
 * S as in enkf_analysis, with the impact factor of observation j on state
 * point i
 *   d = |i - obs_loc[j]|, and on a ring (ring > 0) d = min(d, ring - d);
 *   delta(i, j) = exp(-d / length), and 0 when radius >= 0 and d > radius.
 * (The paper's Lorenz-96 runs: ring = length = n_state, no radius.)
 * obs_loc: DEVICE array of n_obs int64 state indices in [0, n_state) (other
 * values only change the distances). length finite and > 0; ring 0 or >=
 * n_state. Other arguments and errors as enkf_analysis; uses the plan's V
 * and dtype. The n_state x n_obs weighted matrix is never stored: one fused
 * kernel forms its tiles on the matrix cores and applies them to Z.
 * 4 n_state n_obs N flops (S V^T recomputed per 128 columns of X^A when N >
 * 128). Allocates nothing.
 */
enkf_status enkf_localized_analysis(enkf_sm_plan plan, int64_t n_state, const void* XB, int64_t ldx, const void* Z,
                                    int64_t ldz, const int64_t* obs_loc, double length, int64_t radius, int64_t ring,
                                    void* XA, int64_t ldxa);

/*
 * The same analysis update with the ensemble in its own storage type and the
 * n_state x N x N product on a chosen matrix-core input type: x_dtype is the
 * type of XB and XA; math is ENKF_MATH_F64 (x_dtype F64) or ENKF_MATH_F32,
 * ENKF_MATH_BF16, ENKF_MATH_F16, ENKF_MATH_BF16X3, ENKF_MATH_F16X2 (x_dtype
 * F32; accumulation in FP32). G = V^T Z is formed in the plan's storage type
 * with FP64 accumulation. Z is in the plan's dtype. XA must not overlap XB.
 */
enkf_status enkf_analysis_ex(enkf_sm_plan plan, int64_t n_state, enkf_dtype x_dtype, enkf_math math, const void* XB,
                             int64_t ldx, const void* Z, int64_t ldz, void* XA, int64_t ldxa);

/* Synchronise the plan's stream and report the factor's pivots, the last
 * solve's refinement record and any latched device error. */
enkf_status enkf_sm_get_info(enkf_sm_plan plan, enkf_sm_info* info);

/* What ENKF_FLAG_AUTOTUNE measured at init: *count (<= 4) widths and the
 * milliseconds of one factorisation + solve with each (HOST arrays of 4, or
 * NULL). *count = 0 when the plan did not tune (or reused a tuned width). */
enkf_status enkf_sm_get_tuning(enkf_sm_plan plan, int32_t* widths, double* ms, int32_t* count);

/* Copy the pivots gamma_1..gamma_N (FP64, HOST buffer of n_ens entries) and,
 * when pivoting, the level order (HOST int32 buffer or NULL: entry k is the V
 * column used at level k). Synchronises. */
enkf_status enkf_sm_get_pivots(enkf_sm_plan plan, double* gamma_host, int32_t* perm_host);

/*
 * Measurement: when enabled, the plan records a HIP event pair on its stream
 * around every kernel launch it makes and, per kernel class, accumulates the
 * elapsed time, the number of launches and the algorithmic bytes and flops of
 * those launches (the minimum each launch must move or compute; the byte and
 * flop models are stated next to each kernel). Enabling or disabling clears
 * the totals. enkf_sm_get_timing synchronises on the recorded events.
 * Classes: 0 factor level sweeps (plain), 1 solve level sweeps (plain),
 * 2 build, 3 analysis update, 4 split-K products, 5 panel updates (blocked),
 * 6 panel factorisations (blocked), 7 FP64 residuals (refinement),
 * 8 Step 1 (with the plain form's first look-ahead products), 9 level sweeps
 * of a fused factorisation + solve (plain), 10 localized analysis updates,
 * 11 the products G = V^T Z of the FP64 residuals (class 7 is then the
 * residual D - (R Z + V G) itself).
 */
enkf_status enkf_sm_set_timing(enkf_sm_plan plan, int32_t enable);
enkf_status enkf_sm_get_timing(enkf_sm_plan plan, int32_t kernel_class, double* total_ms, int64_t* launches,
                               double* alg_bytes, double* alg_flops);

/* Release the workspace. Synchronises the plan's stream first. */
void enkf_sm_destroy(enkf_sm_plan plan);

/*
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * enkf_sm_init followed by enkf_sm_factor_solve on the same arguments, with
 * the same kernels and launch sequence (so the same Z, bit for bit), but the
 * plan's workspace carved from a static device array of
 * ENKF_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, held until the
 * process ends, instead of hipMalloc. No device memory is allocated or freed.
 *   desc, r, V, ldv: as enkf_sm_init (ENKF_FLAG_AUTOTUNE is refused: the
 *     tuner allocates; block-diagonal R is not available here);
 *   nrhs, D, ldd, Z, ldz, info: as enkf_sm_factor_solve (info != NULL
 *     synchronises `stream` and reports; NULL only enqueues);
 *   stream: hipStream_t as void* (NULL: the null stream).
 * A problem whose workspace (U: n_obs x (n_ens + max_nrhs) in the storage
 * type for the plain algorithm, plus panel and reduction buffers) exceeds
 * the scratch returns ENKF_ERR_NOT_SUPPORTED with the needed size in
 * enkf_last_error_message(). Every call on a GPU shares that GPU's scratch:
 * calls that overlap in time on one GPU (different streams, or host threads)
 * race and give wrong results; calls on one stream are ordered and safe.
 * The factor lives in the scratch only until the next call.
 */
#define ENKF_NOALLOC_SCRATCH_BYTES (64u << 20)
enkf_status enkf_sm_solve_noalloc(const enkf_sm_desc* desc, const double* r, const void* V, int64_t ldv,
                                  int32_t nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz,
                                  enkf_sm_info* info, void* stream);

/*
 * Measured matrix-core throughput of the current device, the on-box
 * counterpart of the published peaks the rooflines divide by (MI355X dense:
 * FP64 78.6, FP32 157.3, BF16/FP16 2500 TFLOP/s). Runs a kernel in which
 * every wave issues 4096 x 8 independent MFMAs on register operands
 * (16x16x4 for F64/F32, 16x16x32 for BF16/F16; no memory traffic) on a
 * private stream, times it with HIP events and stores TFLOP/s in *tflops.
 * math: ENKF_MATH_F64, _F32, _BF16 or _F16 (else ENKF_ERR_NOT_SUPPORTED).
 * Allocates 4 bytes of device memory for the duration of the call.
 */
enkf_status enkf_mfma_peak(enkf_math math, double* tflops);

const char* enkf_status_string(enkf_status s);
/* Detail of the last error raised on the calling thread. */
const char* enkf_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* ENKF_SM_H */
