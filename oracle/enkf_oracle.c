/*
 * FP64 CPU oracle for the EnKF analysis by the iterative Sherman-Morrison
 * formula (Nino-Ruiz, Sandu and Anderson, "An efficient implementation of the
 * ensemble Kalman filter based on an iterative Sherman-Morrison formula").
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header or constant with the GPU library and includes none of its files.
 *
 * Plain, slow and meant to be read against the paper:
 *   - FP64 everywhere, plain loops, no BLAS, built with -ffp-contract=off;
 *   - every dot product sums its index in ascending order;
 *   - OpenMP only spreads independent columns (or independent problems) over
 *     threads; each column is still computed serially, so results do not
 *     depend on the thread count.
 * Matrices are column-major: element (i, j) of an m-row matrix with leading
 * dimension ld sits at [i + j*ld]; one column per ensemble member.
 *
 * Return codes: 0 success, 1 invalid argument, 2 a pivot gamma_k that is not
 * finite or not > 0 (the positive-definiteness premise of Section 3.3 failed),
 * 3 out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define E_ARG 1
#define E_NOT_SPD 2
#define E_NOMEM 3

#define AT(A, ld, i, j) ((A)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

static double dot_col(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Iterative Sherman-Morrison solve S*(R, V, D) of Section 3.1:
 * solves (R + V V^T) Z = D with R = diag(r).
 *
 * Step 1 (eq. SM-step-1):  Z0 = R^{-1} D,  U0 = R^{-1} V   (division by r_i).
 * Step 2 (eq. SM-step-2), for k = 1..N:
 *     gamma_k = 1 + v_k^T u_k^{(k-1)},       h_k = u_k^{(k-1)} / gamma_k,
 *     Z^{(k)}  = Z^{(k-1)} - h_k (v_k^T Z^{(k-1)}),
 *     u_i^{(k)} = u_i^{(k-1)} - h_k (v_k^T u_i^{(k-1)})   for i = k+1..N.
 * u_k is not updated after its own level.
 *
 * n, N     number of observations and of ensemble members (both >= 1)
 * r        (n) diagonal of R, each finite and > 0
 * V        (n x N, ldv) scaled observed anomalies
 * D        (n x nrhs, ldd) right-hand sides (nrhs >= 0; the paper has nrhs = N)
 * Z        (n x nrhs, ldz) output
 * Ufac     optional (n x N, ld n): column k receives u_k^{(k-1)}
 * gamma    optional (N): the pivots gamma_k
 * pivot    0: natural order. 1: Section 3.4 pivoting -- before level k choose
 *          the column i >= k maximising |1 + v_i^T u_i^{(k-1)}| (ties: the
 *          smallest i) and swap columns k and i of V and U.
 * perm     optional (N): perm[k] = original V column used at level k
 * longops  optional: multiplications and divisions performed, the count of
 *          Section 3.2 (3(N^2 n + N n) for nrhs = N without pivoting).
 */
/*
 * Step 1 for a block-diagonal R (Section 2.1: R = diag(R_1, ..., R_B), each
 * R_b an SPD N_b x N_b block; Section 3.1: Z0 = R^{-1} D, U0 = R^{-1} V are
 * formed block by block): Y = R^{-1} X with a dense Cholesky factorisation
 * R_b = L L^T of each block, then L y = x and L^T z = y per column.
 * Block b covers rows off[b] .. off[b+1]-1; its matrix is column-major at
 * Rb + sum_{c<b} N_c^2.
 */
static int block_r_solve(int64_t nblk, const int64_t* off, const double* Rb, const double* X, int64_t ldx,
                         int32_t m, double* Y, int64_t ldy) {
    int64_t roff = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t r0 = off[b], s = off[b + 1] - off[b];
        double* L = (double*)malloc(sizeof(double) * (size_t)(s * s));
        double* y = (double*)malloc(sizeof(double) * (size_t)s);
        if (!L || !y) { free(L); free(y); return E_NOMEM; }
        memcpy(L, Rb + roff, sizeof(double) * (size_t)(s * s));
        for (int64_t j = 0; j < s; ++j) {          /* column-oriented Cholesky */
            double d = L[j + j * s];
            for (int64_t k = 0; k < j; ++k) d -= L[j + k * s] * L[j + k * s];
            if (!(d > 0.0) || !isfinite(d)) { free(L); free(y); return E_NOT_SPD; }
            d = sqrt(d);
            L[j + j * s] = d;
            for (int64_t i = j + 1; i < s; ++i) {
                double v = L[i + j * s];
                for (int64_t k = 0; k < j; ++k) v -= L[i + k * s] * L[j + k * s];
                L[i + j * s] = v / d;
            }
        }
        for (int32_t c = 0; c < m; ++c) {
            for (int64_t i = 0; i < s; ++i) {      /* L y = x */
                double v = AT(X, ldx, r0 + i, c);
                for (int64_t k = 0; k < i; ++k) v -= L[i + k * s] * y[k];
                y[i] = v / L[i + i * s];
            }
            for (int64_t i = s - 1; i >= 0; --i) { /* L^T z = y */
                double v = y[i];
                for (int64_t k = i + 1; k < s; ++k) v -= L[k + i * s] * AT(Y, ldy, r0 + k, c);
                AT(Y, ldy, r0 + i, c) = v / L[i + i * s];
            }
        }
        free(L);
        free(y);
        roff += s * s;
    }
    return OK;
}

static int sm_solve_core(int64_t n, int32_t N, const double* r, int64_t nblk, const int64_t* boff,
                         const double* Rb, const double* V, int64_t ldv, const double* D, int64_t ldd, int32_t nrhs,
                         double* Z, int64_t ldz, double* Ufac, double* gamma, int32_t pivot, int32_t* perm,
                         int64_t* longops);

int oracle_sm_solve(int64_t n, int32_t N, const double* r, const double* V, int64_t ldv,
                    const double* D, int64_t ldd, int32_t nrhs, double* Z, int64_t ldz,
                    double* Ufac, double* gamma, int32_t pivot, int32_t* perm, int64_t* longops) {
    if (!r) return E_ARG;
    return sm_solve_core(n, N, r, 0, NULL, NULL, V, ldv, D, ldd, nrhs, Z, ldz, Ufac, gamma, pivot, perm, longops);
}

/* The same solve with a block-diagonal R (Step 1 by block_r_solve). */
int oracle_sm_solve_block_r(int64_t n, int32_t N, int64_t nblk, const int64_t* boff, const double* Rb,
                            const double* V, int64_t ldv, const double* D, int64_t ldd, int32_t nrhs, double* Z,
                            int64_t ldz, double* gamma) {
    if (nblk < 1 || !boff || !Rb || boff[0] != 0 || boff[nblk] != n) return E_ARG;
    for (int64_t b = 0; b < nblk; ++b)
        if (boff[b + 1] <= boff[b]) return E_ARG;
    return sm_solve_core(n, N, NULL, nblk, boff, Rb, V, ldv, D, ldd, nrhs, Z, ldz, NULL, gamma, 0, NULL, NULL);
}

static int sm_solve_core(int64_t n, int32_t N, const double* r, int64_t nblk, const int64_t* boff,
                         const double* Rb, const double* V, int64_t ldv, const double* D, int64_t ldd, int32_t nrhs,
                         double* Z, int64_t ldz, double* Ufac, double* gamma, int32_t pivot, int32_t* perm,
                         int64_t* longops) {
    if (n < 1 || N < 1 || nrhs < 0 || ldv < n || (nrhs > 0 && (ldd < n || ldz < n))) return E_ARG;
    if (!V || (nrhs > 0 && (!D || !Z))) return E_ARG;
    if (r)
        for (int64_t i = 0; i < n; ++i)
            if (!(r[i] > 0.0) || !isfinite(r[i])) return E_NOT_SPD;

    double* U = (double*)malloc(sizeof(double) * (size_t)n * (size_t)N);
    double* Vw = (double*)malloc(sizeof(double) * (size_t)n * (size_t)N);
    double* h = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* pm = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    if (!U || !Vw || !h || !pm) { free(U); free(Vw); free(h); free(pm); return E_NOMEM; }
    int64_t ops = 0;

    /* Working copy of V whose columns may be permuted by pivoting. */
    for (int32_t j = 0; j < N; ++j) {
        pm[j] = j;
        memcpy(Vw + (size_t)j * n, &AT(V, ldv, 0, j), sizeof(double) * (size_t)n);
    }

    /* Step 1. */
    if (r) {
        #pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < N; ++j)
            for (int64_t i = 0; i < n; ++i) AT(U, n, i, j) = AT(Vw, n, i, j) / r[i];
        #pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < nrhs; ++j)
            for (int64_t i = 0; i < n; ++i) AT(Z, ldz, i, j) = AT(D, ldd, i, j) / r[i];
        ops += n * (int64_t)N + n * (int64_t)nrhs;
    } else {
        int st = block_r_solve(nblk, boff, Rb, Vw, n, N, U, n);
        if (st == OK && nrhs > 0) st = block_r_solve(nblk, boff, Rb, D, ldd, nrhs, Z, ldz);
        if (st != OK) { free(U); free(Vw); free(h); free(pm); return st; }
    }

    int status = OK;
    for (int32_t k = 0; k < N; ++k) {
        if (pivot) {
            /* Section 3.4: evaluate each candidate pivot, then swap. */
            int32_t best = k;
            double best_val = -1.0;
            for (int32_t i = k; i < N; ++i) {
                double g = fabs(1.0 + dot_col(n, &AT(Vw, n, 0, i), &AT(U, n, 0, i)));
                ops += n;
                if (g > best_val) { best_val = g; best = i; }
            }
            if (best != k) {
                for (int64_t i = 0; i < n; ++i) {
                    double t = AT(Vw, n, i, k); AT(Vw, n, i, k) = AT(Vw, n, i, best); AT(Vw, n, i, best) = t;
                    t = AT(U, n, i, k); AT(U, n, i, k) = AT(U, n, i, best); AT(U, n, i, best) = t;
                }
                int32_t t = pm[k]; pm[k] = pm[best]; pm[best] = t;
            }
        }
        const double* vk = &AT(Vw, n, 0, k);
        const double* uk = &AT(U, n, 0, k);
        /* eq. SM-step-2-h */
        double g = 1.0 + dot_col(n, vk, uk);
        ops += n;
        if (!isfinite(g) || !(g > 0.0)) { status = E_NOT_SPD; break; }
        for (int64_t i = 0; i < n; ++i) h[i] = uk[i] / g;
        ops += n;
        if (gamma) gamma[k] = g;
        if (Ufac) memcpy(Ufac + (size_t)k * n, uk, sizeof(double) * (size_t)n);
        /* eq. SM-step-2-Z: every column of Z */
        #pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < nrhs; ++j) {
            double* zj = &AT(Z, ldz, 0, j);
            double c = dot_col(n, vk, zj);
            for (int64_t i = 0; i < n; ++i) zj[i] -= h[i] * c;
        }
        ops += 2 * n * (int64_t)nrhs;
        /* eq. SM-step-2-u: columns k+1..N of U */
        #pragma omp parallel for schedule(static)
        for (int32_t j = k + 1; j < N; ++j) {
            double* uj = &AT(U, n, 0, j);
            double c = dot_col(n, vk, uj);
            for (int64_t i = 0; i < n; ++i) uj[i] -= h[i] * c;
        }
        ops += 2 * n * (int64_t)(N - k - 1);
    }
    if (perm) memcpy(perm, pm, sizeof(int32_t) * (size_t)N);
    if (longops) *longops = ops;
    free(U); free(Vw); free(h); free(pm);
    return status;
}

/*
 * Apply a stored factor to new right-hand sides: Step 1 on X, then the
 * Z-update of every level (eq. SM-step-2-Z) with h_k = Ufac[:,k] / gamma_k.
 * The factor holds no D, so this is the D-dependent half of S*.
 * perm: NULL, or the level order returned by a pivoted solve.
 */
int oracle_sm_apply(int64_t n, int32_t N, const double* r, const double* V, int64_t ldv,
                    const double* Ufac, const double* gamma, const int32_t* perm,
                    const double* X, int64_t ldx, int32_t nrhs, double* Y, int64_t ldy) {
    if (n < 1 || N < 1 || nrhs < 0 || ldv < n || ldx < n || ldy < n) return E_ARG;
    double* h = (double*)malloc(sizeof(double) * (size_t)n);
    if (!h) return E_NOMEM;
    #pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < nrhs; ++j)
        for (int64_t i = 0; i < n; ++i) AT(Y, ldy, i, j) = AT(X, ldx, i, j) / r[i];
    for (int32_t k = 0; k < N; ++k) {
        const double* vk = &AT(V, ldv, 0, perm ? perm[k] : k);
        for (int64_t i = 0; i < n; ++i) h[i] = Ufac[(size_t)k * n + i] / gamma[k];
        #pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < nrhs; ++j) {
            double* yj = &AT(Y, ldy, 0, j);
            double c = dot_col(n, vk, yj);
            for (int64_t i = 0; i < n; ++i) yj[i] -= h[i] * c;
        }
    }
    free(h);
    return OK;
}

/*
 * Residual of the system of eq. EnKSM:system-to-solve-V:
 *   rho = D - (R Z + V (V^T Z)),   computed as G = V^T Z first.
 */
int oracle_residual(int64_t n, int32_t N, const double* r, const double* V, int64_t ldv,
                    const double* Z, int64_t ldz, const double* D, int64_t ldd, int32_t nrhs,
                    double* rho, int64_t ldr) {
    if (n < 1 || N < 1 || nrhs < 0) return E_ARG;
    double* G = (double*)malloc(sizeof(double) * (size_t)N * (size_t)(nrhs > 0 ? nrhs : 1));
    if (!G) return E_NOMEM;
    #pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < nrhs; ++j)
        for (int32_t l = 0; l < N; ++l) G[l + (size_t)j * N] = dot_col(n, &AT(V, ldv, 0, l), &AT(Z, ldz, 0, j));
    #pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < nrhs; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int32_t l = 0; l < N; ++l) s += AT(V, ldv, i, l) * G[l + (size_t)j * N];
            AT(rho, ldr, i, j) = AT(D, ldd, i, j) - (r[i] * AT(Z, ldz, i, j) + s);
        }
    free(G);
    return OK;
}

/*
 * Inputs of the analysis (Section 2 and eq. EnKSM:system-rewritten) from the
 * background ensemble, with H a row selection x -> x[obs_idx]:
 *   xbar = X^B 1 / N                                   (ensemble mean)
 *   V    = H (X^B - xbar 1^T) / sqrt(N - 1)            (eq. EnSM:Matrix-member-deviations, member-observations)
 *   D    = (y 1^T + E) - H X^B                         (perturbed observations; eq. system-rhs)
 */
int oracle_build_vd(int64_t n_state, int32_t N, const double* XB, int64_t ldx, const int64_t* obs_idx,
                    int64_t n_obs, const double* y, const double* E, int64_t lde, double* V, int64_t ldv,
                    double* D, int64_t ldd) {
    if (n_state < 1 || N < 2 || n_obs < 1 || ldx < n_state || lde < n_obs || ldv < n_obs || ldd < n_obs)
        return E_ARG;
    for (int64_t i = 0; i < n_obs; ++i)
        if (obs_idx[i] < 0 || obs_idx[i] >= n_state) return E_ARG;
    const double scale = sqrt((double)(N - 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_obs; ++i) {
        int64_t s = obs_idx[i];
        double sum = 0.0;
        for (int32_t j = 0; j < N; ++j) sum += AT(XB, ldx, s, j);
        double mean = sum / (double)N;
        for (int32_t j = 0; j < N; ++j) {
            AT(V, ldv, i, j) = (AT(XB, ldx, s, j) - mean) / scale;
            AT(D, ldd, i, j) = (y[i] + AT(E, lde, i, j)) - AT(XB, ldx, s, j);
        }
    }
    return OK;
}

/*
 * Analysis update of Section 3.1 (the SMEnKF listing): X^A = X^B + S (V^T Z),
 * S = (X^B - xbar 1^T) / sqrt(N - 1). G = V^T Z is formed first (N x N).
 * XA may not alias XB.
 */
int oracle_analysis(int64_t n_state, int32_t N, int64_t n_obs, const double* XB, int64_t ldx,
                    const double* V, int64_t ldv, const double* Z, int64_t ldz, double* XA, int64_t ldxa) {
    if (n_state < 1 || N < 2 || n_obs < 1) return E_ARG;
    double* G = (double*)malloc(sizeof(double) * (size_t)N * (size_t)N);
    if (!G) return E_NOMEM;
    #pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < N; ++j)
        for (int32_t l = 0; l < N; ++l) G[l + (size_t)j * N] = dot_col(n_obs, &AT(V, ldv, 0, l), &AT(Z, ldz, 0, j));
    const double scale = sqrt((double)(N - 1));
    int fail = 0;
    #pragma omp parallel
    {
        double* dx = (double*)malloc(sizeof(double) * (size_t)N);
        if (!dx) {
            #pragma omp atomic write
            fail = 1;
        }
        #pragma omp for schedule(static)
        for (int64_t s = 0; s < n_state; ++s) {
            if (!dx) continue;
            double sum = 0.0;
            for (int32_t j = 0; j < N; ++j) sum += AT(XB, ldx, s, j);
            double mean = sum / (double)N;
            for (int32_t l = 0; l < N; ++l) dx[l] = (AT(XB, ldx, s, l) - mean) / scale;
            for (int32_t j = 0; j < N; ++j) {
                double acc = 0.0;
                for (int32_t l = 0; l < N; ++l) acc += dx[l] * G[l + (size_t)j * N];
                AT(XA, ldxa, s, j) = AT(XB, ldx, s, j) + acc;
            }
        }
        free(dx);
    }
    free(G);
    return fail ? E_NOMEM : OK;
}

/*
 * Partial localization (Section 3.1.2, eq. localized-correction-component):
 *   XA[i, l] = XB[i, l] + sum_k S[i, k] sum_j delta(i, j) V[j, k] Z[j, l],
 *   S = (XB - mean_row(XB)) / sqrt(N - 1),
 * with the impact factor of observation j (located at state index loc[j]) on
 * state point i
 *   d = |i - loc[j]|, on a ring of `ring` points d = min(d, ring - d);
 *   delta(i, j) = exp(-d / length), or 0 when radius >= 0 and d > radius
 * (the paper's Lorenz-96 experiments: ring = length = n_state, no radius).
 * Written in the formula's order: for each (i, l), the outer sum over k of
 * S[i, k] times the inner sum over j. O(n_state N^2 n_obs) work.
 * oracle_localized_rows computes the rows [row_begin, row_end) only (the
 * rows are independent); the others of XA are not written.
 */
static double impact(int64_t i, int64_t loc, double length, int64_t radius, int64_t ring) {
    int64_t d = i > loc ? i - loc : loc - i;
    if (ring > 0 && ring - d < d) d = ring - d;
    if (radius >= 0 && d > radius) return 0.0;
    return exp(-(double)d / length);
}

int oracle_localized_rows(int64_t n_state, int32_t N, int64_t n_obs, const double* XB, int64_t ldx,
                          const double* V, int64_t ldv, const double* Z, int64_t ldz, const int64_t* loc,
                          double length, int64_t radius, int64_t ring, int64_t row_begin, int64_t row_end,
                          double* XA, int64_t ldxa) {
    if (n_state < 1 || N < 2 || n_obs < 1 || !(length > 0.0)) return E_ARG;
    if (row_begin < 0 || row_end > n_state || row_begin > row_end) return E_ARG;
    for (int64_t j = 0; j < n_obs; ++j)
        if (loc[j] < 0 || loc[j] >= n_state) return E_ARG;
    const double scale = sqrt((double)(N - 1));
    int fail = 0;
    #pragma omp parallel
    {
        double* S = (double*)malloc(sizeof(double) * (size_t)N);
        double* dl = (double*)malloc(sizeof(double) * (size_t)n_obs);
        if (!S || !dl) {
            #pragma omp atomic write
            fail = 1;
        }
        #pragma omp for schedule(dynamic, 4)
        for (int64_t i = row_begin; i < row_end; ++i) {
            if (!S || !dl) continue;
            double sum = 0.0;
            for (int32_t k = 0; k < N; ++k) sum += AT(XB, ldx, i, k);
            const double mean = sum / (double)N;
            for (int32_t k = 0; k < N; ++k) S[k] = (AT(XB, ldx, i, k) - mean) / scale;
            for (int64_t j = 0; j < n_obs; ++j) dl[j] = impact(i, loc[j], length, radius, ring);
            for (int32_t l = 0; l < N; ++l) {
                double outer = 0.0;
                for (int32_t k = 0; k < N; ++k) {
                    double inner = 0.0;
                    for (int64_t j = 0; j < n_obs; ++j) inner += dl[j] * AT(V, ldv, j, k) * AT(Z, ldz, j, l);
                    outer += S[k] * inner;
                }
                AT(XA, ldxa, i, l) = AT(XB, ldx, i, l) + outer;
            }
        }
        free(S);
        free(dl);
    }
    return fail ? E_NOMEM : OK;
}

/* Every row of the partially localized update. */
int oracle_localized_analysis(int64_t n_state, int32_t N, int64_t n_obs, const double* XB, int64_t ldx,
                              const double* V, int64_t ldv, const double* Z, int64_t ldz, const int64_t* loc,
                              double length, int64_t radius, int64_t ring, double* XA, int64_t ldxa) {
    return oracle_localized_rows(n_state, N, n_obs, XB, ldx, V, ldv, Z, ldz, loc, length, radius, ring, 0, n_state,
                                 XA, ldxa);
}

/*
 * Localized analyses, one independent small problem each. Problem p uses the
 * observations win_start[p], win_start[p]+1, ..., win_start[p]+win_len[p]-1,
 * taken modulo n_glob (a cyclic domain), i.e. the rows of the global r, V, D;
 * it solves its local system with oracle_sm_solve and updates the single state
 * point state_idx[p]:
 *   xa[p, :] = X^B[s, :] + S[s, :] (V_p^T Z_p),   s = state_idx[p].
 * xa is (n_prob x N), leading dimension ldxa (>= n_prob).
 */
int oracle_local_analysis(int64_t n_glob, int32_t N, const double* r, const double* V, int64_t ldv,
                          const double* D, int64_t ldd, int64_t n_state, const double* XB, int64_t ldx,
                          int64_t n_prob, const int64_t* win_start, const int64_t* win_len,
                          const int64_t* state_idx, double* xa, int64_t ldxa) {
    if (n_glob < 1 || N < 2 || n_prob < 0 || ldxa < n_prob) return E_ARG;
    for (int64_t p = 0; p < n_prob; ++p)
        if (win_len[p] < 1 || win_len[p] > n_glob || win_start[p] < 0 || win_start[p] >= n_glob ||
            state_idx[p] < 0 || state_idx[p] >= n_state)
            return E_ARG;
    int status = OK;
    const double scale = sqrt((double)(N - 1));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_prob; ++p) {
        int64_t m = win_len[p];
        double* buf = (double*)malloc(sizeof(double) * ((size_t)m * (3 * (size_t)N + 1) + 2 * (size_t)N * N));
        if (!buf) {
            #pragma omp atomic write
            status = E_NOMEM;
            continue;
        }
        double *rl = buf, *Vl = rl + m, *Dl = Vl + (size_t)m * N, *Zl = Dl + (size_t)m * N;
        double *G = Zl + (size_t)m * N, *dx = G + (size_t)N * N;
        for (int64_t i = 0; i < m; ++i) {
            int64_t g = (win_start[p] + i) % n_glob;
            rl[i] = r[g];
            for (int32_t j = 0; j < N; ++j) {
                Vl[i + (size_t)j * m] = AT(V, ldv, g, j);
                Dl[i + (size_t)j * m] = AT(D, ldd, g, j);
            }
        }
        int st = oracle_sm_solve(m, N, rl, Vl, m, Dl, m, N, Zl, m, NULL, NULL, 0, NULL, NULL);
        if (st != OK) {
            #pragma omp atomic write
            status = st;
        } else {
            for (int32_t j = 0; j < N; ++j)
                for (int32_t l = 0; l < N; ++l) G[l + (size_t)j * N] = dot_col(m, Vl + (size_t)l * m, Zl + (size_t)j * m);
            int64_t s = state_idx[p];
            double sum = 0.0;
            for (int32_t j = 0; j < N; ++j) sum += AT(XB, ldx, s, j);
            double mean = sum / (double)N;
            for (int32_t l = 0; l < N; ++l) dx[l] = (AT(XB, ldx, s, l) - mean) / scale;
            for (int32_t j = 0; j < N; ++j) {
                double acc = 0.0;
                for (int32_t l = 0; l < N; ++l) acc += dx[l] * G[l + (size_t)j * N];
                AT(xa, ldxa, p, j) = AT(XB, ldx, s, j) + acc;
            }
        }
        free(buf);
    }
    return status;
}

/*
 * Lorenz-96 forecast (the model of the Lorenz-96 experiments, Section 4):
 *   dx_i/dt = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F,  indices cyclic,
 * advanced by the classical fourth-order Runge-Kutta method with step dt,
 *   k1 = f(x), k2 = f(x + dt/2 k1), k3 = f(x + dt/2 k2), k4 = f(x + dt k3),
 *   x <- x + dt/6 (k1 + 2 k2 + 2 k3 + k4),
 * nsteps times, for each of the m columns of X (n x m, ldx). n >= 4.
 */
static void l96_f(int64_t n, const double* x, double F, double* f) {
    for (int64_t i = 0; i < n; ++i) {
        const double xp1 = x[(i + 1) % n], xm1 = x[(i + n - 1) % n], xm2 = x[(i + n - 2) % n];
        f[i] = (xp1 - xm2) * xm1 - x[i] + F;
    }
}

int oracle_l96_rk4(int64_t n, int64_t m, double* X, int64_t ldx, int64_t nsteps, double F, double dt) {
    if (n < 4 || m < 0 || ldx < n || nsteps < 0) return E_ARG;
    int fail = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        double* w = (double*)malloc(sizeof(double) * (size_t)n * 5);
        if (!w) {
            #pragma omp atomic write
            fail = 1;
            continue;
        }
        double *k1 = w, *k2 = w + n, *k3 = w + 2 * n, *k4 = w + 3 * n, *y = w + 4 * n;
        double* x = X + j * ldx;
        for (int64_t s = 0; s < nsteps; ++s) {
            l96_f(n, x, F, k1);
            for (int64_t i = 0; i < n; ++i) y[i] = x[i] + 0.5 * dt * k1[i];
            l96_f(n, y, F, k2);
            for (int64_t i = 0; i < n; ++i) y[i] = x[i] + 0.5 * dt * k2[i];
            l96_f(n, y, F, k3);
            for (int64_t i = 0; i < n; ++i) y[i] = x[i] + dt * k3[i];
            l96_f(n, y, F, k4);
            for (int64_t i = 0; i < n; ++i) x[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        }
        free(w);
    }
    return fail ? E_NOMEM : OK;
}
