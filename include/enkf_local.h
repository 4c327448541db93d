/*
 * enkf_local.h -- batched localized EnKF analyses on one MI355X (gfx950).
 *
 * Many independent small analyses, one per state point, each using only the
 * observations of its own window, run in one kernel launch (captured once
 * into a HIP graph and replayed). Problem p:
 *   rows g = (win_start[p] + i) mod n_glob, i = 0 .. win_len[p]-1, of the
 *   global r, V, D (a cyclic domain);
 *   Z_p = (R_p + V_p V_p^T)^{-1} D_p        (Section 3, eq. system-to-solve-V)
 *   xa_p = x^B_s + S_s (V_p^T Z_p),  s = state_idx[p],
 *   S_s = (x^B_s - mean(x^B_s)) / sqrt(N-1)  (Section 3.1, the SMEnKF update,
 *   for the single state row s).
 * Each local solve is the Sherman-Morrison-Woodbury form (eq. SWM) with one
 * panel of all N levels: M_p = I + V_p^T R_p^{-1} V_p = L D L^T, whose
 * pivots D are the gamma_k of the iterative formula (Section 3.3), and
 * V_p^T Z_p = M_p^{-1} V_p^T R_p^{-1} D_p, so that
 * xa_p = x^B_s + (R_p^{-1} V_p y)^T D_p / sqrt(N-1) with y = M_p^{-1} delta_s,
 * delta_s the centred ensemble row of X^B at s. The Gram product
 * V_p^T R_p^{-1} V_p runs on FP32 matrix cores (FP32 storage) with FP64
 * accumulation across row stages; the pivots, the N x N solve and the second
 * pass over the window forming (R_p^{-1} V_p y)^T D_p are FP64 arithmetic.
 *
 * Overlapping windows (ENKF_LOCAL_PATH_PREFIX): the window sums
 * A_p = V_p^T R_p^{-1} V_p and Q_p = V_p^T R_p^{-1} D_p are differences of
 * FP64 prefix sums over the ring at 16-row chunk boundaries plus the at most
 * 30 rows outside them, and xa_p = x^B_s + y^T Q_p / sqrt(N-1) (the same
 * identity); all sums, the N x N factorization and the solves are FP64
 * arithmetic on the FP32 inputs. A row whose r is not finite and > 0, or
 * whose V or D entries are not finite, is left out of the prefix sums; a
 * window containing one takes its rows one by one (so such a row affects
 * exactly the windows that contain it, as on the streaming path).
 *
 * Conventions as in enkf_sm.h: column-major, device pointers, stream-ordered,
 * enkf_status returns; argument errors are found on the host.
 */
#ifndef ENKF_LOCAL_H
#define ENKF_LOCAL_H

#include <stdint.h>

#include "enkf_sm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ENKF_LOCAL_MAX_ENS 64   /* N <= 64 */

/* enkf_local_desc.tune */
#define ENKF_LOCAL_TUNE_DEFAULT 0  /* the prefix path when its workspace fits and the windows hold at least
                                      n_glob rows in all, else the streaming kernel's default configuration */
#define ENKF_LOCAL_TUNE_TIME    1  /* time both paths (and the streaming configurations) on the first call */
#define ENKF_LOCAL_TUNE_STREAM  2  /* the streaming kernel only */
#define ENKF_LOCAL_TUNE_PREFIX  3  /* the prefix path only (ENKF_ERR_NOT_SUPPORTED at init when it does not fit) */

/* enkf_local_get_path */
#define ENKF_LOCAL_PATH_STREAM 0   /* one pass over each window per problem (one kernel) */
#define ENKF_LOCAL_PATH_PREFIX 1   /* chunk sums, their prefix scan, then one wave per problem (three kernels) */

typedef struct {
    int64_t n_glob;   /* observations on the cyclic domain (rows of r, V, D), >= 1 */
    int32_t n_ens;    /* N, 2 <= N <= ENKF_LOCAL_MAX_ENS */
    int64_t n_state;  /* rows of X^B */
    int64_t n_prob;   /* number of local problems, >= 0 */
    int32_t tune;     /* ENKF_LOCAL_TUNE_*; other values return ENKF_ERR_INVALID_ARG */
} enkf_local_desc;

typedef struct enkf_local_plan_s* enkf_local_plan;

/*
 * Create a plan for a fixed set of windows. win_start, win_len and state_idx
 * are HOST arrays of n_prob entries (copied): 0 <= win_start < n_glob,
 * 1 <= win_len <= n_glob, 0 <= state_idx < n_state; violations return
 * ENKF_ERR_INVALID_ARG. The plan orders the problems longest-first and deals
 * them to the blocks of the launch (a static schedule). Allocates (the prefix
 * path's workspace: (ceil(n_glob / 16) + 1) (2 N'N + 2) doubles, N' = N rounded
 * up to even, when that is at most 1 GiB); the stream is fixed here.
 */
enkf_status enkf_local_init(enkf_local_plan* out, const enkf_local_desc* desc, const int64_t* win_start,
                            const int64_t* win_len, const int64_t* state_idx, void* stream);

/*
 * Run every local analysis. r (n_glob, FP64, > 0), V and D (n_glob x N, FP32,
 * leading dimension ldv), XB (n_state x N, FP32, ldx), XA (n_prob x N, FP32,
 * ldxa >= n_prob): row p receives xa_p. gamma (FP64, n_prob x N, leading
 * dimension n_prob) receives the pivots of every problem, or is NULL.
 * One HIP graph replay (one kernel on the streaming path, three on the
 * prefix path); allocates nothing. A pivot that is not finite or not > 0, or
 * an r_i in a window that is not finite and > 0, latches ENKF_ERR_NOT_SPD,
 * reported by enkf_local_sync.
 */
enkf_status enkf_local_analysis(enkf_local_plan plan, const double* r, const float* V, const float* D, int64_t ldv,
                                const float* XB, int64_t ldx, float* XA, int64_t ldxa, double* gamma);

/* Synchronise the plan's stream and return any latched device error.
 * *rows_per_stage and *blocks receive the configuration in use (may be NULL):
 * on the prefix path 0 and n_prob (one wave per problem). */
enkf_status enkf_local_sync(enkf_local_plan plan, int32_t* rows_per_stage, int32_t* blocks);

/* The path in use (ENKF_LOCAL_PATH_*); after a tuned plan's first analysis,
 * the one the timing chose. Host only. */
enkf_status enkf_local_get_path(enkf_local_plan plan, int32_t* path);

void enkf_local_destroy(enkf_local_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* ENKF_LOCAL_H */
