/*
 * Seeded synthetic inputs for the EnKF analysis workloads.
 *
 * This file holds no part of the analysis method. It only produces the
 * arrays that both the HIP path and the FP64 oracle consume:
 *   - a counter-based random stream (Philox4x64-10, Salmon, Moraes, Dror and
 *     Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) turned into
 *     uniforms and, by the Box-Muller transform, standard normals;
 *   - the Lorenz-96 model (the cyclic ring of the paper's Lorenz-96 section,
 *     forcing F) advanced by the classical four-stage Runge-Kutta scheme.
 *
 * Every value depends only on (seed, purpose, index), never on the number of
 * threads, so the same arrays come out on any host.
 * Built with gcc -O2 -fopenmp -ffp-contract=off.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

/* One Philox4x64-10 block: 4 words of output for a 4-word counter and a
 * 2-word key. */
void synth_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        __uint128_t p0 = (__uint128_t)PHILOX_M0 * c0;
        __uint128_t p1 = (__uint128_t)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform strictly inside (0, 1). */
static inline double u01(uint64_t x) {
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Words of stream (seed, purpose): block b uses counter (b+1, 0, 0, 0) and key
 * (seed, purpose), the same convention as numpy's Philox bit generator. */
static inline void block_words(uint64_t seed, uint64_t purpose, uint64_t b, uint64_t w[4]) {
    uint64_t ctr[4] = {b + 1, 0, 0, 0};
    uint64_t key[2] = {seed, purpose};
    synth_philox4x64(ctr, key, w);
}

/* out[i] = uniform #(offset+i) of the stream, scaled to [lo, hi). */
void synth_uniform(uint64_t seed, uint64_t purpose, int64_t offset, int64_t count,
                   double lo, double hi, double* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t idx = (uint64_t)(offset + i);
        uint64_t w[4];
        block_words(seed, purpose, idx >> 2, w);
        out[i] = lo + (hi - lo) * u01(w[idx & 3]);
    }
}

/* out[i] = standard normal #(offset+i) of the stream. Each Philox block gives
 * two Box-Muller pairs. */
void synth_normal(uint64_t seed, uint64_t purpose, int64_t offset, int64_t count, double* out) {
    const double two_pi = 6.283185307179586476925286766559;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t idx = (uint64_t)(offset + i);
        uint64_t w[4];
        block_words(seed, purpose, idx >> 2, w);
        int pair = (int)((idx >> 1) & 1);
        double a = u01(w[2 * pair]), b = u01(w[2 * pair + 1]);
        double rad = sqrt(-2.0 * log(a));
        out[i] = (idx & 1) ? rad * sin(two_pi * b) : rad * cos(two_pi * b);
    }
}

/* Integer draws uniform on [lo, hi] (inclusive), by rejection-free scaling of
 * a 53-bit uniform (bias below 2^-40 for the small ranges used here). */
void synth_randint(uint64_t seed, uint64_t purpose, int64_t offset, int64_t count,
                   int64_t lo, int64_t hi, int64_t* out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t idx = (uint64_t)(offset + i);
        uint64_t w[4];
        block_words(seed, purpose, idx >> 2, w);
        double u = u01(w[idx & 3]);
        int64_t v = lo + (int64_t)floor(u * (double)(hi - lo + 1));
        out[i] = v > hi ? hi : v;
    }
}

/* Lorenz-96 tendency with cyclic indexing:
 * f_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F. */
static void l96_tendency(int64_t n, const double* x, double F, double* f, int par) {
    #pragma omp parallel for schedule(static) if (par)
    for (int64_t i = 0; i < n; ++i) {
        int64_t ip1 = (i + 1 == n) ? 0 : i + 1;
        int64_t im1 = (i == 0) ? n - 1 : i - 1;
        int64_t im2 = (i >= 2) ? i - 2 : i - 2 + n;
        f[i] = (x[ip1] - x[im2]) * x[im1] - x[i] + F;
    }
}

/* Classical RK4 for one state vector; `par` selects threading inside. */
static void l96_rk4(int64_t n, double* x, double F, double dt, int64_t nsteps, int par,
                    double* k1, double* k2, double* k3, double* k4, double* tmp) {
    for (int64_t s = 0; s < nsteps; ++s) {
        l96_tendency(n, x, F, k1, par);
        #pragma omp parallel for schedule(static) if (par)
        for (int64_t i = 0; i < n; ++i) tmp[i] = x[i] + 0.5 * dt * k1[i];
        l96_tendency(n, tmp, F, k2, par);
        #pragma omp parallel for schedule(static) if (par)
        for (int64_t i = 0; i < n; ++i) tmp[i] = x[i] + 0.5 * dt * k2[i];
        l96_tendency(n, tmp, F, k3, par);
        #pragma omp parallel for schedule(static) if (par)
        for (int64_t i = 0; i < n; ++i) tmp[i] = x[i] + dt * k3[i];
        l96_tendency(n, tmp, F, k4, par);
        #pragma omp parallel for schedule(static) if (par)
        for (int64_t i = 0; i < n; ++i)
            x[i] = x[i] + (dt / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
}

/* Advance one state in place (threads split the ring). Returns 0, or 1 when
 * scratch cannot be allocated. */
int synth_l96_advance(int64_t n, double* x, double F, double dt, int64_t nsteps) {
    double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)n);
    if (!buf) return 1;
    l96_rk4(n, x, F, dt, nsteps, 1, buf, buf + n, buf + 2 * n, buf + 3 * n, buf + 4 * n);
    free(buf);
    return 0;
}

/* Advance every column of X (n x m, column-major, leading dimension ldx) in
 * place; threads take whole members, each integrated serially, so the result
 * does not depend on the thread count. */
int synth_l96_advance_members(int64_t n, int64_t m, double* X, int64_t ldx, double F, double dt,
                              int64_t nsteps) {
    int nt = omp_get_max_threads();
    double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)n * (size_t)nt);
    if (!buf) return 1;
    #pragma omp parallel num_threads(nt)
    {
        double* b = buf + (size_t)omp_get_thread_num() * 5 * (size_t)n;
        #pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < m; ++j)
            l96_rk4(n, X + j * ldx, F, dt, nsteps, 0, b, b + n, b + 2 * n, b + 3 * n, b + 4 * n);
    }
    free(buf);
    return 0;
}
