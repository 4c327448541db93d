// Batched localized analyses (enkf_local.h), gfx950.
//
// One launch runs every local problem. Blocks take statically scheduled
// lists of problems (longest window first, dealt to the least-loaded block).
// Per problem, 256 threads:
//  1. one streaming pass over the window's rows forms
//       A = (R^{-1} V_p)^T V_p
//     on FP32 matrix cores (16x16x4), the next stage of rows prefetched into
//     registers meanwhile; the FP32 accumulators are emptied into FP64 after
//     every stage;
//  2. M = I + A = L D L^T in FP64 registers (upper blocks of a 16 x 16
//     thread grid, one rank-4 update per four levels), with the forward
//     elimination of delta, the centred ensemble row of the state point,
//     carried along; the pivots D are the gamma_k of the iterative formula
//     (Section 3.3);
//  3. y = M^{-1} delta by the backward substitution (one wave, four rows at
//     a time);
//  4. since V_p^T Z_p = M^{-1} (R^{-1} V_p)^T D_p (the Woodbury form of
//     eq. SWM with one panel), the centre-point update (Section 3.1) is
//     xa = x^B_s + (R^{-1} V_p y)^T D_p / sqrt(N-1), formed by a second,
//     O(n_p N) pass over the window.
// The ensemble is padded to 64 members (zero anomalies give identity rows of
// M and zero products).
#include <algorithm>
#include <cmath>
#include <queue>
#include <type_traits>
#include <vector>

#include "enkf_internal.h"
#include "enkf_local.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int LN = ENKF_LOCAL_MAX_ENS;
constexpr int LT = 256;
constexpr int LDM = LN + 1;

struct LocalArgs {
  int64_t n_glob;
  int N;
  int64_t ldv, ldx, ldxa, n_prob;
  const double* r;
  const float* V;
  const float* D;
  const float* XB;
  float* XA;
  double* gamma;
  const int64_t* win_start;
  const int64_t* win_len;
  const int64_t* state_idx;
  const int32_t* sched;
  const int32_t* sched_off;
  unsigned* status;
  double inv_sqrt;
};

// 1/x to within a few ulp: the hardware estimate refined by two Newton steps
// (each squares the relative error of the estimate).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// Lane k's value of a double (k uniform across the wave).
__device__ __forceinline__ double rdlane(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// O32: every element of V and D lies within 4 GiB of its base, so the row
// offsets are formed in 32 bits (one offset register serves V and D).
template <int KC, bool O32>
__global__ __launch_bounds__(LT, KC == 32 ? 3 : 2) void local_kernel(LocalArgs a) {
  constexpr int LDK = KC + 4;                     // float rows of the Gram stages (16-byte aligned)
  constexpr int PER = LN * KC / LT;               // Gram: staged elements per thread
  constexpr int CSTEP = LT / KC;                  // Gram: column step of a thread's elements
  constexpr int K4 = 64;                          // rows per stage of the second pass (one per lane)
  constexpr int PER4 = LN / 4;                    // second pass: members per thread
  constexpr int LD4D = K4 + 1;                    // rows of the final transposition
  constexpr size_t PH1 = 2 * sizeof(float) * LN * LDK;
  constexpr size_t PH2 = sizeof(double) * (LN * LDM + 8 * LN + 2 * LN);
  constexpr size_t PH4 = sizeof(double) * (LN * LD4D + 2 * 4 * K4 + 4 * LN);
  constexpr size_t SM = PH1 > PH2 ? (PH1 > PH4 ? PH1 : PH4) : (PH2 > PH4 ? PH2 : PH4);
  __shared__ __attribute__((aligned(16))) char smem[SM];
  __shared__ float xbuf[LN];                       // x^B of the state point (0 past N)
  __shared__ double yv[LN];                        // y = M^{-1} delta (0 past N)
  __shared__ double zv[LN];                        // delta under forward elimination
  __shared__ double zf[LN];                        // z = L^{-1} delta
  // phase 1: Vr[col][k] = V[g_k, col] / r_{g_k} and Vt = V (rows k of the
  // stage); phase 2: M (then the columns of L D), the panels, the pivots and
  // their reciprocals; phase 4: partial sums
  float* Vr = reinterpret_cast<float*>(smem);
  float* Vt = Vr + LN * LDK;
  double* Msh = reinterpret_cast<double*>(smem);
  double* pan = Msh + LN * LDM;                    // [2][4][LN] panels of four columns
  double* piv = pan + 8 * LN;                      // the LN pivots
  double* ipiv = piv + LN;                         // their reciprocals
  double* ored = reinterpret_cast<double*>(smem);  // [LN][LD4D] lane sums of s_i D_i
  double* wpart = ored + LN * LD4D;                // [2][4][K4] partial dots V_i . y
  double* opart = wpart + 2 * 4 * K4;              // [4][LN]
  const int t = threadIdx.x, l = t % 64, w = t / 64;
  const int kk = t % KC, c0 = t / KC;             // Gram: this thread's stage row and first column
  const int beg = a.sched_off[blockIdx.x], end = a.sched_off[blockIdx.x + 1];
  uint32_t coff[O32 ? PER : 1];                   // byte offsets of this thread's Gram columns (O32)
  uint32_t coff4[O32 ? PER4 : 1];                 // and of its second-pass columns
  if constexpr (O32) {
#pragma unroll
    for (int j = 0; j < PER; ++j) coff[j] = (uint32_t)(min(c0 + CSTEP * j, a.N - 1) * a.ldv) * 4u;
#pragma unroll
    for (int j = 0; j < PER4; ++j) coff4[j] = (uint32_t)(min(w + 4 * j, a.N - 1) * a.ldv) * 4u;
  }
  // element (g, column c) of V or D, c the thread's j-th column of a pass
  auto ld = [&](const float* base, int64_t g, int c, uint32_t off) -> float {
    if constexpr (O32)
      return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + ((uint32_t)g * 4u + off));
    else
      return base[g + (int64_t)min(c, a.N - 1) * a.ldv];
  };
  for (int q = beg; q < end; ++q) {
    const int p = a.sched[q];
    const int64_t g0 = a.win_start[p], m = a.win_len[p], s = a.state_idx[p];
    auto row_of = [&](int64_t i) -> int64_t {     // global row of window row i (clamped to the window)
      int64_t g = g0 + min(i, m - 1);
      return g >= a.n_glob ? g - a.n_glob : g;
    };

    // 1. A = (R^{-1} V_p)^T V_p over the window. The next stage is loaded
    //    into registers (branch-free: rows past the window and members past
    //    N read valid elements and are zeroed when staged) while the matrix
    //    cores work on the current one. Wave w forms rows 16w .. 16w+15.
    mf_f4 acc[4];
    double wide[4][4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      acc[tj] = mf_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) wide[tj][r] = 0.0;
    }
    float vreg[PER];
    double rreg;
    auto fetch = [&](int64_t i0) {
      const int64_t g = row_of(i0 + kk);
      rreg = a.r[g];
#pragma unroll
      for (int j = 0; j < PER; ++j) vreg[j] = ld(a.V, g, c0 + CSTEP * j, O32 ? coff[j] : 0u);
    };
    auto stash = [&](int64_t i0) {
      const bool row_ok = i0 + kk < m;
      if (row_ok && (!(rreg > 0.0) || !__builtin_isfinite(rreg))) atomicOr(a.status, kStatusNotSpd);
      const double rinv = row_ok ? 1.0 / rreg : 0.0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int c = c0 + CSTEP * j;
        const float v = (row_ok && c < a.N) ? vreg[j] : 0.f;
        Vt[c * LDK + kk] = v;
        Vr[c * LDK + kk] = (float)((double)v * rinv);
      }
    };
    __syncthreads();                               // the previous problem is done with the LDS
    const float xs = (w == 0 && l < a.N) ? a.XB[s + (int64_t)l * a.ldx] : 0.f;   // x^B_s, used at the end
    fetch(0);
    stash(0);
    if (w == 0) xbuf[l] = xs;
    __syncthreads();
    for (int64_t i0 = 0; i0 < m; i0 += KC) {
      fetch(i0 + KC);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k4 = 0; k4 < KC; k4 += 4) {
        const float aop = Vr[(16 * w + l % 16) * LDK + k4 + l / 16];
        float bop[4];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) bop[tj] = Vt[(16 * tj + l % 16) * LDK + k4 + l / 16];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) acc[tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop[tj], acc[tj], 0, 0, 0);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
        for (int r = 0; r < 4; ++r) wide[tj][r] += (double)acc[tj][r];
        acc[tj] = mf_f4{0.f, 0.f, 0.f, 0.f};
      }
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      stash(i0 + KC);                             // after the last stage: zeros, unused
      __syncthreads();
    }
    // 2. M = I + A to the LDS, redistributed to a 16 x 16 thread grid: thread
    //    (gi, gj) keeps the elements (gi + 16 r, gj + 16 c), c >= r, of the
    //    upper blocks. Right-looking M = L D L^T four levels at a time: the
    //    panel P of columns k0 .. k0+3 (published in the LDS) has the diagonal
    //    block P_d = L4 D4 L4^T; every kept element takes
    //    M -= (L4^{-1} P_i)^T D4^{-1} (L4^{-1} P_j), which equals the four
    //    single-level updates c c^T / d; D4 holds the pivots gamma_k0 ..
    //    gamma_k0+3 of the iterative formula (Section 3.3) and L4^{-1} P_i the
    //    columns of L D. Elements of finished rows take rounding-size values
    //    no step reads.
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + 4 * (l / 16) + r;
        const int col = 16 * tj + l % 16;
        Msh[row * LDM + col] = wide[tj][r] + (row == col ? 1.0 : 0.0);
      }
    __syncthreads();
    const int gi = t % 16, gj = t / 16;
    double mv[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = r; c < 4; ++c) mv[r][c] = Msh[(gi + 16 * r) * LDM + gj + 16 * c];
    pan[(t / LN) * LN + t % LN] = Msh[(t / LN) * LDM + t % LN];   // panel 0 = rows 0..3
    if (w == 0) {                                  // delta, the centred ensemble row of the state point
      const double x = (double)xbuf[l];
      const double mean = wsum(x) / (double)a.N;
      zv[l] = (l < a.N) ? x - mean : 0.0;
    }
    __syncthreads();
    auto ldl_phase = [&](auto kb_c) {
      constexpr int KB = decltype(kb_c)::value;
#pragma unroll 1
      for (int ss = 0; ss < 4; ++ss) {
        const int k0 = 16 * KB + 4 * ss;
        const double* P = pan + (ss & 1) * 4 * LN;
        double* Pn = pan + ((ss + 1) & 1) * 4 * LN;
        double Lm[4][4], dv[4], iv[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          double e = P[qq * LN + k0 + qq];
#pragma unroll
          for (int u = 0; u < qq; ++u) e -= Lm[qq][u] * Lm[qq][u] * dv[u];
          dv[qq] = e;
          iv[qq] = recip(e);
#pragma unroll
          for (int v = qq + 1; v < 4; ++v) {
            double f = P[qq * LN + k0 + v];
#pragma unroll
            for (int u = 0; u < qq; ++u) f -= Lm[v][u] * Lm[qq][u] * dv[u];
            Lm[v][qq] = f * iv[qq];
          }
        }
        double ch[4][4];                           // rows: L4^{-1} P_i (then scaled by D4^{-1})
#pragma unroll
        for (int r = KB; r < 4; ++r)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            double x = P[qq * LN + gi + 16 * r];
#pragma unroll
            for (int u = 0; u < qq; ++u) x -= Lm[qq][u] * ch[r][u];
            ch[r][qq] = x;
          }
        if (gj == 0)                               // columns k0..k0+3 of L D
#pragma unroll
          for (int r = KB; r < 4; ++r)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) Msh[(k0 + qq) * LDM + gi + 16 * r] = ch[r][qq];
#pragma unroll
        for (int r = KB; r < 4; ++r)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) ch[r][qq] *= iv[qq];
        // forward elimination of delta: the panel's entries become
        // L4^{-1} delta_P (final entries of z = L^{-1} delta); later rows take
        // the same rank-4 update as M
        double zh[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          double v = zv[k0 + qq];
#pragma unroll
          for (int u = 0; u < qq; ++u) v -= Lm[qq][u] * zh[u];
          zh[qq] = v;
        }
        if (gj == 0) {
#pragma unroll
          for (int r = KB; r < 4; ++r) {
            const int i = gi + 16 * r;
            double v = zv[i];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) v -= ch[r][qq] * zh[qq];
            if (r > KB || i > k0 + 3) zv[i] = v;
          }
        }
        if (t == 0)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) zf[k0 + qq] = zh[qq];
#pragma unroll
        for (int c = KB; c < 4; ++c) {             // column block c: L4^{-1} P_j, then its elements
          double cj[4];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            double x = P[qq * LN + gj + 16 * c];
#pragma unroll
            for (int u = 0; u < qq; ++u) x -= Lm[qq][u] * cj[u];
            cj[qq] = x;
          }
#pragma unroll
          for (int r = KB; r <= c; ++r)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) mv[r][c] -= ch[r][qq] * cj[qq];
        }
        if (t == 0)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            piv[k0 + qq] = dv[qq];
            ipiv[k0 + qq] = iv[qq];
          }
        const int qn = gi - (k0 + 4) % 16;         // next panel: rows k0+4 .. k0+7
        if (k0 + 4 < LN && qn >= 0 && qn < 4) {
          if (ss < 3) {
#pragma unroll
            for (int c = KB; c < 4; ++c) Pn[qn * LN + gj + 16 * c] = mv[KB][c];
          } else {
            if constexpr (KB < 3) {
#pragma unroll
              for (int c = KB + 1; c < 4; ++c) Pn[qn * LN + gj + 16 * c] = mv[KB + 1][c];
            }
          }
        }
        __syncthreads();
      }
    };
    ldl_phase(std::integral_constant<int, 0>{});
    ldl_phase(std::integral_constant<int, 1>{});
    ldl_phase(std::integral_constant<int, 2>{});
    ldl_phase(std::integral_constant<int, 3>{});
    if (t < a.N) {
      const double d = piv[t];
      if (a.gamma) a.gamma[p + (int64_t)t * a.n_prob] = d;
      if (!(d > 0.0) || !__builtin_isfinite(d)) atomicOr(a.status, kStatusNotSpd);
    }
    // 3. y = M^{-1} delta = L^{-T} D^{-1} z with z = L^{-1} delta from the
    //    factorization, four rows at a time (wave 0, lane i holds entry i;
    //    L[i][k] = Msh[k][i] / d_k for i > k).
    if (w == 0) {
      double y = zf[l] * ipiv[l];                 // D^{-1} z, then y = L^{-T} (D^{-1} z)
#pragma unroll 2
      for (int k0 = LN - 4; k0 >= 0; k0 -= 4) {
        double yp[4];
#pragma unroll
        for (int qq = 3; qq >= 0; --qq) {
          double v = rdlane(y, k0 + qq);
#pragma unroll
          for (int u = qq + 1; u < 4; ++u) v -= Msh[(k0 + qq) * LDM + k0 + u] * ipiv[k0 + qq] * yp[u];
          yp[qq] = v;
        }
        double acc_y = 0.0;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) acc_y += Msh[l * LDM + k0 + qq] * yp[qq];
        const int dq = l - k0;
        const double yin = dq == 0 ? yp[0] : dq == 1 ? yp[1] : dq == 2 ? yp[2] : yp[3];
        y = (l < k0) ? y - acc_y * ipiv[l] : (dq <= 3 ? yin : y);
      }
      yv[l] = (l < a.N) ? y : 0.0;
    }
    // 4. V_p^T Z_p = M^{-1} (R^{-1} V_p)^T D_p (the Woodbury form of eq. SWM
    //    with one panel), so the centre-point update of the SMEnKF
    //    (Section 3.1) is xa = x^B_s + (R^{-1} V_p y)^T D_p / sqrt(N-1): a
    //    second pass over the window, 64 rows a stage, lane = row and wave w
    //    = members w, w + 4, ...: s_i = (V_i . y) / r_i from the four waves'
    //    partial dots, then every lane accumulates s_i D_i over its members
    //    (FP64 arithmetic on the FP32 rows); one transposition through the
    //    LDS sums the lanes at the end.
    float v4[PER4], d4[PER4];
    double r4;
    auto fetch4 = [&](int64_t i0) {
      const int64_t g = row_of(i0 + l);
      r4 = a.r[g];
#pragma unroll
      for (int j = 0; j < PER4; ++j) {
        v4[j] = ld(a.V, g, w + 4 * j, O32 ? coff4[j] : 0u);
        d4[j] = ld(a.D, g, w + 4 * j, O32 ? coff4[j] : 0u);
      }
    };
    fetch4(0);
    __syncthreads();                               // y is complete; the LDS is free
    double yr[PER4], o4[PER4];
#pragma unroll
    for (int j = 0; j < PER4; ++j) {
      yr[j] = yv[w + 4 * j];
      o4[j] = 0.0;
    }
    int buf = 0;
    for (int64_t i0 = 0; i0 < m; i0 += K4) {
      const bool row_ok = i0 + l < m;
      double wp = 0.0;                             // members past N: y = 0
#pragma unroll
      for (int j = 0; j < PER4; ++j) wp += (double)v4[j] * yr[j];
      wpart[(buf * 4 + w) * K4 + l] = wp;
      float dn[PER4];
#pragma unroll
      for (int j = 0; j < PER4; ++j) dn[j] = d4[j];
      const double rinv = row_ok ? 1.0 / r4 : 0.0;
      fetch4(i0 + K4);                             // past the window: clamped rows, unused
      __syncthreads();
      const double* wb = wpart + buf * 4 * K4;
      const double sr = ((wb[l] + wb[K4 + l]) + (wb[2 * K4 + l] + wb[3 * K4 + l])) * rinv;
#pragma unroll
      for (int j = 0; j < PER4; ++j) o4[j] += sr * (double)dn[j];
      buf ^= 1;
    }
    __syncthreads();                               // the last partials are read
#pragma unroll
    for (int j = 0; j < PER4; ++j) ored[(w + 4 * j) * LD4D + l] = o4[j];
    __syncthreads();
    {
      double part = 0.0;                           // member l, lanes 16w .. 16w+15
#pragma unroll
      for (int i = 16 * w; i < 16 * w + 16; ++i) part += ored[l * LD4D + i];
      opart[w * LN + l] = part;
    }
    __syncthreads();
    if (w == 0 && l < a.N) {
      const double part = (opart[l] + opart[LN + l]) + (opart[2 * LN + l] + opart[3 * LN + l]);
      a.XA[p + (int64_t)l * a.ldxa] = (float)((double)xbuf[l] + part * a.inv_sqrt);
    }
  }
}

const void* kernel_for(int kc, bool o32) {
  if (o32)
    return kc == 64 ? reinterpret_cast<const void*>(&local_kernel<64, true>)
                    : reinterpret_cast<const void*>(&local_kernel<32, true>);
  return kc == 64 ? reinterpret_cast<const void*>(&local_kernel<64, false>)
                  : reinterpret_cast<const void*>(&local_kernel<32, false>);
}

// ------------------------------------------------------------------ overlapping windows
// Windows are contiguous runs of the ring, and neighbouring windows share
// most of their rows. Every window sum the analysis needs,
//   A_p = V_p^T R_p^{-1} V_p   and   Q_p = V_p^T R_p^{-1} D_p,
// is a difference of prefix sums over the ring taken at CH-row chunk
// boundaries (FP64), plus the window's rows before its first and after its
// last boundary (at most 2 (CH - 1) rows), so no problem streams its whole
// window. With y = M_p^{-1} delta_s (M_p = I + A_p), the centre-point update
// is xa = x^B_s + y^T Q_p / sqrt(N-1), the same Woodbury form as above.
// Rows whose r_g is not finite and > 0, or whose V or D entries are not
// finite, add nothing to the chunk sums and are counted instead; a window
// whose boundary range holds such a row takes all of its rows directly, so
// it sees them exactly as the streaming kernel does.
constexpr int CH = 16;                            // rows per chunk

struct PrefixArgs {
  int64_t n_glob;
  int N, Np, nc;                                  // Np: N rounded up to even
  int64_t ldv;
  int64_t W;                                      // doubles per prefix entry: 2 Np N sums, the bad-row count, one pad
  const double* r;
  const float* V;
  const float* D;
  double* pre;                                    // (nc + 1) entries of W doubles
};

// Entry layout: A at [0, Np N), Q at [Np N, 2 Np N), element (i, j) of either
// at ((i / 2) N + j) 2 + i % 2, so lane j reads rows i, i + 1 of its column
// as one 16-byte load and a wave's loads are contiguous; the bad-row count at
// 2 Np N.
__device__ __forceinline__ int64_t pre_index(int i, int j, int N) { return ((int64_t)(i >> 1) * N + j) * 2 + (i & 1); }

// Block c writes the sums of chunk c (rows [c CH, min((c + 1) CH, n_glob)))
// into entry c.
__global__ __launch_bounds__(256) void local_chunk_kernel(PrefixArgs a) {
  __shared__ __attribute__((aligned(16))) double vs[CH][LN];    // v_g
  __shared__ __attribute__((aligned(16))) double ws[CH][LN];    // v_g / r_g
  __shared__ __attribute__((aligned(16))) double dsh[CH][LN];   // d_g
  __shared__ int bad[CH];
  const int t = threadIdx.x, c = blockIdx.x;
  const int64_t g0 = (int64_t)c * CH;
  const int nr = (int)min<int64_t>(CH, a.n_glob - g0);
  const int rho = t % CH, q = t / CH;             // row of the chunk; members q + 16 u
  if (t < CH) bad[t] = 0;
  __syncthreads();
  const bool rok = rho < nr;
  const int64_t g = g0 + (rok ? rho : 0);
  const double rr = a.r[g];
  bool fine = rr > 0.0 && __builtin_isfinite(rr);
  double v[LN / 16], d[LN / 16];
#pragma unroll
  for (int u = 0; u < LN / 16; ++u) {
    const int i = q + 16 * u;
    v[u] = (rok && i < a.N) ? (double)a.V[g + (int64_t)i * a.ldv] : 0.0;
    d[u] = (rok && i < a.N) ? (double)a.D[g + (int64_t)i * a.ldv] : 0.0;
    fine = fine && __builtin_isfinite(v[u]) && __builtin_isfinite(d[u]);
  }
  if (rok && !fine) bad[rho] = 1;
  __syncthreads();
  const bool use = rok && !bad[rho];
  const double ri = use ? 1.0 / rr : 0.0;
#pragma unroll
  for (int u = 0; u < LN / 16; ++u) {
    const int i = q + 16 * u;
    vs[rho][i] = use ? v[u] : 0.0;
    ws[rho][i] = use ? v[u] * ri : 0.0;
    dsh[rho][i] = use ? d[u] : 0.0;
  }
  __syncthreads();
  // thread t: rows i0 .. i0+3, columns j0 + 16 y (y < 4) of both sums (rows
  // past the chunk are zero), so that 16 lanes store 16 consecutive columns
  // of a row pair: 256 contiguous bytes
  double* out = a.pre + (int64_t)c * a.W;
  const int half = a.Np * a.N;
  const int i0 = 4 * (t / 16), j0 = t % 16;
  double sa[4][4], sq[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) sa[x][y] = sq[x][y] = 0.0;
#pragma unroll 2
  for (int k = 0; k < CH; ++k) {
    double vi[4], wi[4], wj[4], dj[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      vi[x] = vs[k][i0 + x];
      wi[x] = ws[k][i0 + x];
      wj[x] = ws[k][j0 + 16 * x];
      dj[x] = dsh[k][j0 + 16 * x];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        sa[x][y] = fma(vi[x], wj[y], sa[x][y]);
        sq[x][y] = fma(wi[x], dj[y], sq[x][y]);
      }
  }
#pragma unroll
  for (int x = 0; x < 4; x += 2)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + x, j = j0 + 16 * y;      // rows i, i + 1 of column j: one 16-byte store
      if (i < a.Np && j < a.N) {
        *reinterpret_cast<double2*>(out + pre_index(i, j, a.N)) = double2{sa[x][y], sa[x + 1][y]};
        *reinterpret_cast<double2*>(out + half + pre_index(i, j, a.N)) = double2{sq[x][y], sq[x + 1][y]};
      }
    }
  if (t == 0) {
    int nb = 0;
    for (int k = 0; k < nr; ++k) nb += bad[k];
    out[2 * half] = (double)nb;
    out[2 * half + 1] = 0.0;
  }
}

// In place: entry c becomes the sum of chunks < c (entry 0 = 0) and entry nc
// the sum of all. Thread (e, seg) of a block takes position e of the entries
// of its segment of chunks; the segments' totals are combined in order.
constexpr int SCAN_SEG = 16;
__global__ __launch_bounds__(256) void local_scan_kernel(PrefixArgs a) {
  __shared__ double tot[SCAN_SEG][16];
  const int el = threadIdx.x % 16, seg = threadIdx.x / 16;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  const int L = (a.nc + SCAN_SEG - 1) / SCAN_SEG;
  const int c0 = min(seg * L, a.nc), c1 = min(c0 + L, a.nc);
  const bool ok = e < a.W;
  constexpr int B = 16;                           // loads in flight per thread
  double v[B];
  double s = 0.0;
  if (ok)
    for (int cb = c0; cb < c1; cb += B) {
#pragma unroll
      for (int u = 0; u < B; ++u) v[u] = cb + u < c1 ? a.pre[(int64_t)(cb + u) * a.W + e] : 0.0;
#pragma unroll
      for (int u = 0; u < B; ++u) s += v[u];
    }
  tot[seg][el] = s;
  __syncthreads();
  double run = 0.0;
  for (int k = 0; k < seg; ++k) run += tot[k][el];
  if (ok) {
    for (int cb = c0; cb < c1; cb += B) {
      if (cb != c0 || c1 - c0 > B) {             // more than one batch: load this one again
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = cb + u < c1 ? a.pre[(int64_t)(cb + u) * a.W + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (cb + u < c1) {
          a.pre[(int64_t)(cb + u) * a.W + e] = run;
          run += v[u];
        }
    }
    if (seg == SCAN_SEG - 1) a.pre[(int64_t)a.nc * a.W + e] = run;
  }
}

// A block's window, decomposed on the host: at most three boundary terms
// (prefix entries with signs), at most two edge ranges of fewer than CH rows
// each, and the window's runs of the ring for the direct path.
struct WinPlan {
  int64_t st;                                     // state point
  int64_t ea[2], eb[2];                           // edge ranges [ea, eb)
  int64_t sa[2], sb[2];                           // the window's runs [sa, sb)
  int32_t p, nt, ne, nseg;                        // problem, terms, edge ranges, runs
  int32_t tc[3], sg[3];                           // prefix entries and signs (unused: entry 0, sign 0)
  int32_t pad[4];
};
static_assert(sizeof(WinPlan) == 128, "WinPlan layout");

// One wave per problem: lane j holds column j of M_p in FP64 registers.
// Every load the window needs before the factorization (its edge rows, the
// boundary terms of A_p, the bad-row counts, x^B_s) is issued up front; the
// edge rows stay in the LDS for the Q_p phase.
__global__ __launch_bounds__(64) void local_prefix_kernel(LocalArgs a, PrefixArgs pa, const WinPlan* wpl) {
  __shared__ __attribute__((aligned(16))) float vsh[2][CH][LN];
  __shared__ __attribute__((aligned(16))) float dsh[2][CH][LN];
  __shared__ double rsh[2][CH];
  __shared__ double ssh[CH];
  __shared__ double ysh[LN];
  const int l = threadIdx.x;
  const int N = a.N;
  const WinPlan& w = wpl[blockIdx.x];
  const int p = w.p, nt = w.nt, ne = w.ne;
  const int rho = l % CH, q = l / CH;             // staging: row rho, members q + 4 u

  // rows [g0, g0 + nr) of r, V (and D) into registers, then into slot sl:
  // lane (rho, q) takes row rho
  struct Rows {
    float v[LN / 4], d[LN / 4];
    double rr;
    bool rok;
  };
  auto fetch = [&](Rows& x, int64_t g0, int nr, bool with_d) {
    x.rok = rho < nr;
    const int64_t g = g0 + (x.rok ? rho : 0);
#pragma unroll
    for (int u = 0; u < LN / 4; ++u) {         // clamped addresses, unused values masked to +0 (no branch)
      const int i = q + 4 * u;
      const int64_t off = g + (int64_t)min(i, N - 1) * a.ldv;
      const unsigned keep = (x.rok && i < N) ? ~0u : 0u;
      x.v[u] = __uint_as_float(__float_as_uint(a.V[off]) & keep);
      x.d[u] = with_d ? __uint_as_float(__float_as_uint(a.D[off]) & keep) : 0.f;
    }
    x.rr = a.r[g];
  };
  auto put = [&](const Rows& x, int sl, bool with_d) {
    if (q == 0) {
      if (x.rok && !(x.rr > 0.0 && __builtin_isfinite(x.rr))) atomicOr(a.status, kStatusNotSpd);
      rsh[sl][rho] = x.rok ? 1.0 / x.rr : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LN / 4; ++u) {
      vsh[sl][rho][q + 4 * u] = x.v[u];
      if (with_d) dsh[sl][rho][q + 4 * u] = x.d[u];
    }
  };
  auto stage = [&](int sl, int64_t g0, int nr, bool with_d) {
    Rows x;
    fetch(x, g0, nr, with_d);
    put(x, sl, with_d);
  };
  // col[i] += v_ri v_rj / r_r over the rows of slot sl
  double col[LN];
  auto gram = [&](int sl, int nr) {
    for (int r = 0; r < nr; ++r) {
      const double wj = (double)vsh[sl][r][l] * rsh[sl][r];
#pragma unroll
      for (int i = 0; i < LN; i += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(&vsh[sl][r][i]);
        col[i] = fma((double)v4.x, wj, col[i]);
        col[i + 1] = fma((double)v4.y, wj, col[i + 1]);
        col[i + 2] = fma((double)v4.z, wj, col[i + 2]);
        col[i + 3] = fma((double)v4.w, wj, col[i + 3]);
      }
    }
  };
  // col[i] = sum_k sg_k P_{tc_k}[part][i][l] (column l of the window sum;
  // unused terms read entry 0, which is zero, with sign 0)
  auto terms = [&](int64_t part) {
    const double* E0 = pa.pre + (int64_t)w.tc[0] * pa.W + part;
    const double* E1 = pa.pre + (int64_t)w.tc[1] * pa.W + part;
    const double* E2 = pa.pre + (int64_t)w.tc[2] * pa.W + part;
    const double s0 = w.sg[0], s1 = w.sg[1], s2 = w.sg[2];
#pragma unroll
    for (int i2 = 0; i2 < LN / 2; ++i2) {
      if (2 * i2 < N) {
        const int64_t o = pre_index(2 * i2, l, N);
        const double2 v0 = *reinterpret_cast<const double2*>(E0 + o);
        const double2 v1 = *reinterpret_cast<const double2*>(E1 + o);
        double2 v2 = {0.0, 0.0};
        if (nt > 2) v2 = *reinterpret_cast<const double2*>(E2 + o);
        col[2 * i2] = fma(s2, v2.x, fma(s1, v1.x, s0 * v0.x));
        col[2 * i2 + 1] = fma(s2, v2.y, fma(s1, v1.y, s0 * v0.y));
      }
    }
  };

  const int64_t cnt_off = 2 * (int64_t)pa.Np * N;
  double nbad = 0.0;
  for (int k = 0; k < nt; ++k) nbad += (double)w.sg[k] * pa.pre[(int64_t)w.tc[k] * pa.W + cnt_off];
  const double xs = l < N ? (double)a.XB[w.st + (int64_t)l * a.ldx] : 0.0;
  {
    Rows e0, e1;                                  // both edge ranges' loads in flight together
    fetch(e0, w.ea[0], ne > 0 ? (int)(w.eb[0] - w.ea[0]) : 0, true);
    fetch(e1, w.ea[1], ne > 1 ? (int)(w.eb[1] - w.ea[1]) : 0, true);
    put(e0, 0, true);
    put(e1, 1, true);
  }
#pragma unroll
  for (int i = 0; i < LN; ++i) col[i] = 0.0;
  if (l < N && nt > 0) terms(0);
  __syncthreads();
  for (int k = 0; k < ne; ++k) gram(k, (int)(w.eb[k] - w.ea[k]));
  const bool direct = nbad > 0.5;                 // a bad row in the boundary range: every row directly
  if (direct) {
#pragma unroll
    for (int i = 0; i < LN; ++i) col[i] = 0.0;
    for (int k = 0; k < w.nseg; ++k)
      for (int64_t g0 = w.sa[k]; g0 < w.sb[k]; g0 += CH) {
        const int nr = (int)min<int64_t>(CH, w.sb[k] - g0);
        __syncthreads();
        stage(0, g0, nr, false);
        __syncthreads();
        gram(0, nr);
      }
  }
#pragma unroll
  for (int i = 0; i < LN; ++i) col[i] += i == l ? 1.0 : 0.0;
  const double mean = wsum(xs) / (double)N;
  double dz = l < N ? xs - mean : 0.0;

  // M = L D L^T, right-looking, one level per step: column k of the current
  // Schur complement is read lane by lane (lane i's entry k, by symmetry)
  // into scalar registers; lane j > k subtracts M[i][k] M[k][j] / d_k from
  // its entries i > k and the forward elimination of delta rides along.
  // Afterwards lane j holds d_k L[j][k] in entry k < j, d_j in entry j and
  // d_j L[i][j] in entries i > j; the pivots d_k are the gamma_k of the
  // iterative formula. Members past N are identity columns with zero delta:
  // their steps change nothing (d = 1, no multiplier), so every step runs
  // without a branch.
  double pivm = 1.0, invm = 1.0;
#pragma unroll
  for (int k = 0; k < LN; ++k) {
    const double d = rdlane(col[k], k);
    const double id = recip(d);
    pivm = l == k ? d : pivm;
    invm = l == k ? id : invm;
    const double tj = l > k ? col[k] * id : 0.0;
    dz = fma(-tj, rdlane(dz, k), dz);
#pragma unroll
    for (int i = k + 1; i < LN; ++i) col[i] = fma(-rdlane(col[k], i), tj, col[i]);
  }
  // y = L^{-T} D^{-1} z: lane i, once y_k (k > i) is known, subtracts
  // L[k][i] y_k = (its entry k / d_i) y_k
  double yv = dz * invm;
#pragma unroll
  for (int k = LN - 1; k >= 0; --k) {
    const double lk = l < k ? col[k] * invm : 0.0;
    yv = fma(-lk, rdlane(yv, k), yv);
  }
  ysh[l] = l < N ? yv : 0.0;
  __syncthreads();

  // out_j = sum_i y_i Q_p[i][j]: boundary terms (column j of their
  // combination first, into the registers of M) and the edge rows,
  // s_g = (v_g . y) / r_g, out_j += s_g d_gj
  double out = 0.0;
  auto qrows = [&](int sl, int nr) {
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < LN / 4; ++u) part = fma((double)vsh[sl][rho][q + 4 * u], ysh[q + 4 * u], part);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (q == 0) ssh[rho] = part * rsh[sl][rho];
    __syncthreads();
    for (int r = 0; r < nr; ++r) out = fma(ssh[r], (double)dsh[sl][r][l], out);
    __syncthreads();
  };
  if (!direct) {
    if (l < N && nt > 0) {
      terms((int64_t)pa.Np * N);
#pragma unroll
      for (int i = 0; i < LN; ++i) out = fma(ysh[i], col[i], out);
    }
    for (int k = 0; k < ne; ++k) qrows(k, (int)(w.eb[k] - w.ea[k]));
  } else {
    for (int k = 0; k < w.nseg; ++k)
      for (int64_t g0 = w.sa[k]; g0 < w.sb[k]; g0 += CH) {
        const int nr = (int)min<int64_t>(CH, w.sb[k] - g0);
        stage(0, g0, nr, true);
        __syncthreads();
        qrows(0, nr);
      }
  }
  if (l < N) {
    a.XA[p + (int64_t)l * a.ldxa] = (float)(xs + out * a.inv_sqrt);
    if (a.gamma) a.gamma[p + (int64_t)l * a.n_prob] = pivm;
    if (!(pivm > 0.0) || !__builtin_isfinite(pivm)) atomicOr(a.status, kStatusNotSpd);
  }
}

}  // namespace

// ------------------------------------------------------------------ plan
struct LocalPlan {
  enkf_local_desc desc{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int64_t* win_start = nullptr;
  int64_t* win_len = nullptr;
  int64_t* state_idx = nullptr;
  int32_t* sched = nullptr;
  int32_t* sched_off = nullptr;
  unsigned* status = nullptr;
  std::vector<int64_t> len_h;
  int n_cu = 256;
  int max_blocks = 0;
  int kc = 32;
  bool o32 = true;
  int nblocks = 0;
  const void* graph_func = nullptr;
  bool tuned = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  LocalArgs args{};
  // overlapping-window path: prefix entries, and the problems in window
  // order dealt to the eight XCDs in contiguous ranges (block b runs on XCD
  // b mod 8, so neighbouring windows share that XCD's L2)
  int path = ENKF_LOCAL_PATH_STREAM;
  bool prefix_ok = false;
  double* pre = nullptr;
  int32_t* psched = nullptr;
  WinPlan* wplan = nullptr;                       // per block of the prefix path
  PrefixArgs pargs{};
  hipGraphNode_t pnode[2] = {nullptr, nullptr};   // chunk sums, scan

  enkf_status set_config(int kc_, int blocks_per_cu);
  enkf_status init_prefix(const int64_t* win_start, const int64_t* state_idx_h);
  enkf_status launch_direct();
  enkf_status build_graph();
  enkf_status set_graph_params();
  const void* main_func() const {
    return path == ENKF_LOCAL_PATH_PREFIX ? reinterpret_cast<const void*>(&local_prefix_kernel) : kernel_for(kc, o32);
  }
  ~LocalPlan();
};

LocalPlan::~LocalPlan() {
  if (stream || ws) (void)hipStreamSynchronize(stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ws) (void)hipFree(ws);
  if (pre) (void)hipFree(pre);
  if (wplan) (void)hipFree(wplan);
}

// Longest-processing-time-first schedule over `nb` blocks; cost of a problem
// is its window length plus a fixed charge for the N x N factorisation.
enkf_status LocalPlan::set_config(int kc_, int blocks_per_cu) {
  const int64_t P = desc.n_prob;
  int nb = (int)std::min<int64_t>(std::max<int64_t>(P, 1), (int64_t)n_cu * blocks_per_cu);
  std::vector<int32_t> order(P);
  for (int64_t i = 0; i < P; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return len_h[x] > len_h[y]; });
  typedef std::pair<int64_t, int> LB;
  std::priority_queue<LB, std::vector<LB>, std::greater<LB>> heap;
  for (int b = 0; b < nb; ++b) heap.push({0, b});
  std::vector<std::vector<int32_t>> lists(nb);
  for (int32_t pidx : order) {
    LB top = heap.top();
    heap.pop();
    lists[top.second].push_back(pidx);
    // cost in row-stage units: the streamed rows (whole stages) plus the
    // factorization and solves, which take about as long as 5 LN rows
    heap.push({top.first + (len_h[pidx] + kc_ - 1) / kc_ * kc_ + 5 * LN, top.second});
  }
  std::vector<int32_t> flat;
  std::vector<int32_t> off(nb + 1, 0);
  flat.reserve(P);
  for (int b = 0; b < nb; ++b) {
    flat.insert(flat.end(), lists[b].begin(), lists[b].end());
    off[b + 1] = (int32_t)flat.size();
  }
  if (P > 0) ENKF_HIP_CHECK(hipMemcpyAsync(sched, flat.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipMemcpyAsync(sched_off, off.data(), sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  kc = kc_;
  nblocks = nb;
  return ENKF_SUCCESS;
}

// Workspace of the overlapping-window path (when it fits) and its problem
// order: sorted by window start, dealt in contiguous ranges to the XCDs.
constexpr size_t kMaxPrefixBytes = size_t(1) << 30;
enkf_status LocalPlan::init_prefix(const int64_t* win_start, const int64_t* state_idx_h) {
  const int64_t P = desc.n_prob;
  const int64_t nc = (desc.n_glob + CH - 1) / CH;
  const int Np = (desc.n_ens + 1) & ~1;
  const int64_t W = 2 * (int64_t)Np * desc.n_ens + 2;
  const double bytes = 8.0 * (double)(nc + 1) * (double)W;
  if (nc > 0x7fffffff || bytes > (double)kMaxPrefixBytes) return ENKF_SUCCESS;
  if (hipMalloc(&pre, (size_t)bytes) != hipSuccess) {
    pre = nullptr;
    (void)hipGetLastError();
    return ENKF_SUCCESS;
  }
  if (hipMalloc(&wplan, sizeof(WinPlan) * (size_t)P) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(pre);
    pre = nullptr;
    wplan = nullptr;
    return ENKF_SUCCESS;
  }
  std::vector<int32_t> order(P);
  for (int64_t i = 0; i < P; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return win_start[x] < win_start[y]; });
  std::vector<int32_t> ps(P);
  int64_t base[9] = {0};
  for (int x = 0; x < 8; ++x) base[x + 1] = base[x] + (P - x + 7) / 8;   // blocks b < P with b mod 8 == x
  for (int64_t b = 0; b < P; ++b) ps[b] = order[base[b % 8] + b / 8];
  // each block's window: runs of the ring, boundary terms, edge ranges
  const int64_t n = desc.n_glob;
  std::vector<WinPlan> wp(P);
  for (int64_t b = 0; b < P; ++b) {
    const int32_t p = ps[b];
    WinPlan w{};
    w.p = p;
    w.st = state_idx_h[p];
    const int64_t s0 = win_start[p], e0 = s0 + len_h[p];
    w.sa[0] = s0;
    w.sb[0] = std::min(e0, n);
    w.nseg = 1;
    if (e0 > n) {
      w.sa[1] = 0;
      w.sb[1] = e0 - n;
      w.nseg = 2;
    }
    auto bnd = [&](int64_t c) { return std::min(c * CH, n); };
    for (int k = 0; k < w.nseg; ++k) {
      const int64_t lo = w.sa[k], hi = w.sb[k];
      const int64_t c0 = (lo + CH - 1) / CH, c1 = hi == n ? nc : hi / CH;
      if (c0 <= c1) {
        if (c1 != c0) {
          w.tc[w.nt] = (int32_t)c1;
          w.sg[w.nt++] = 1;
          if (c0 != 0) {
            w.tc[w.nt] = (int32_t)c0;
            w.sg[w.nt++] = -1;
          }
        }
        if (lo < bnd(c0)) {
          w.ea[w.ne] = lo;
          w.eb[w.ne++] = bnd(c0);
        }
        if (bnd(c1) < hi) {
          w.ea[w.ne] = bnd(c1);
          w.eb[w.ne++] = hi;
        }
      } else {
        w.ea[w.ne] = lo;
        w.eb[w.ne++] = hi;
      }
    }
    if (w.nt > 3 || w.ne > 2) return fail(ENKF_ERR_NOT_SUPPORTED, "local_init: window decomposition");
    for (int k = 0; k < w.ne; ++k)
      if (w.eb[k] - w.ea[k] > CH || w.eb[k] <= w.ea[k]) return fail(ENKF_ERR_NOT_SUPPORTED, "local_init: edge range");
    wp[b] = w;
  }
  ENKF_HIP_CHECK(hipMemcpyAsync(psched, ps.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipMemcpyAsync(wplan, wp.data(), sizeof(WinPlan) * P, hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  pargs.n_glob = desc.n_glob;
  pargs.N = desc.n_ens;
  pargs.Np = Np;
  pargs.nc = (int)nc;
  pargs.W = W;
  pargs.pre = pre;
  prefix_ok = true;
  return ENKF_SUCCESS;
}

enkf_status LocalPlan::launch_direct() {
  if (path == ENKF_LOCAL_PATH_PREFIX) {
    args.sched = psched;
    hipLaunchKernelGGL(local_chunk_kernel, dim3(pargs.nc), dim3(256), 0, stream, pargs);
    ENKF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(local_scan_kernel, dim3((unsigned)((pargs.W + 15) / 16)), dim3(256), 0, stream, pargs);
    ENKF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(local_prefix_kernel, dim3((unsigned)desc.n_prob), dim3(64), 0, stream, args, pargs,
                       (const WinPlan*)wplan);
    ENKF_HIP_CHECK(hipGetLastError());
    return ENKF_SUCCESS;
  }
  args.sched = sched;
  hipLaunchKernelGGL(reinterpret_cast<void (*)(LocalArgs)>(const_cast<void*>(kernel_for(kc, o32))), dim3(nblocks),
                     dim3(LT), 0, stream, args);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status LocalPlan::build_graph() {
  if (exec) {
    (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  if (graph) {
    (void)hipGraphDestroy(graph);
    graph = nullptr;
  }
  ENKF_HIP_CHECK(hipGraphCreate(&graph, 0));
  hipKernelNodeParams kp{};
  kp.sharedMemBytes = 0;
  kp.extra = nullptr;
  graph_func = main_func();
  if (path == ENKF_LOCAL_PATH_PREFIX) {
    args.sched = psched;
    void* pk_args[] = {&pargs};
    kp.kernelParams = pk_args;
    kp.blockDim = dim3(256);
    kp.func = reinterpret_cast<void*>(&local_chunk_kernel);
    kp.gridDim = dim3(pargs.nc);
    ENKF_HIP_CHECK(hipGraphAddKernelNode(&pnode[0], graph, nullptr, 0, &kp));
    kp.func = reinterpret_cast<void*>(&local_scan_kernel);
    kp.gridDim = dim3((unsigned)((pargs.W + 15) / 16));
    ENKF_HIP_CHECK(hipGraphAddKernelNode(&pnode[1], graph, &pnode[0], 1, &kp));
    const WinPlan* wpp = wplan;
    void* kargs[] = {&args, &pargs, &wpp};
    kp.kernelParams = kargs;
    kp.func = const_cast<void*>(graph_func);
    kp.gridDim = dim3((unsigned)desc.n_prob);
    kp.blockDim = dim3(64);
    ENKF_HIP_CHECK(hipGraphAddKernelNode(&node, graph, &pnode[1], 1, &kp));
  } else {
    args.sched = sched;
    void* kargs[] = {&args};
    kp.kernelParams = kargs;
    kp.func = const_cast<void*>(graph_func);
    kp.gridDim = dim3(nblocks);
    kp.blockDim = dim3(LT);
    ENKF_HIP_CHECK(hipGraphAddKernelNode(&node, graph, nullptr, 0, &kp));
  }
  ENKF_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  return ENKF_SUCCESS;
}

// New data pointers for the nodes of the instantiated graph.
enkf_status LocalPlan::set_graph_params() {
  hipKernelNodeParams kp{};
  kp.sharedMemBytes = 0;
  kp.extra = nullptr;
  if (path == ENKF_LOCAL_PATH_PREFIX) {
    args.sched = psched;
    void* pk_args[] = {&pargs};
    kp.kernelParams = pk_args;
    kp.blockDim = dim3(256);
    kp.func = reinterpret_cast<void*>(&local_chunk_kernel);
    kp.gridDim = dim3(pargs.nc);
    ENKF_HIP_CHECK(hipGraphExecKernelNodeSetParams(exec, pnode[0], &kp));
    kp.func = reinterpret_cast<void*>(&local_scan_kernel);
    kp.gridDim = dim3((unsigned)((pargs.W + 15) / 16));
    ENKF_HIP_CHECK(hipGraphExecKernelNodeSetParams(exec, pnode[1], &kp));
    const WinPlan* wpp = wplan;
    void* kargs[] = {&args, &pargs, &wpp};
    kp.kernelParams = kargs;
    kp.func = const_cast<void*>(main_func());
    kp.gridDim = dim3((unsigned)desc.n_prob);
    kp.blockDim = dim3(64);
    ENKF_HIP_CHECK(hipGraphExecKernelNodeSetParams(exec, node, &kp));
    return ENKF_SUCCESS;
  }
  args.sched = sched;
  void* kargs[] = {&args};
  kp.kernelParams = kargs;
  kp.func = const_cast<void*>(main_func());
  kp.gridDim = dim3(nblocks);
  kp.blockDim = dim3(LT);
  ENKF_HIP_CHECK(hipGraphExecKernelNodeSetParams(exec, node, &kp));
  return ENKF_SUCCESS;
}

}  // namespace enkf

using namespace enkf;

extern "C" {

enkf_status enkf_local_init(enkf_local_plan* out, const enkf_local_desc* d, const int64_t* win_start,
                            const int64_t* win_len, const int64_t* state_idx, void* stream) {
  if (!out || !d) return fail(ENKF_ERR_INVALID_ARG, "local_init: NULL argument");
  *out = nullptr;
  if (d->n_glob < 1 || d->n_state < 1 || d->n_prob < 0) return fail(ENKF_ERR_INVALID_ARG, "local_init: bad sizes");
  if (d->n_ens < 2 || d->n_ens > LN) return fail(ENKF_ERR_INVALID_ARG, "local_init: n_ens outside [2, 64]");
  if (d->n_prob > 0x7fffffff) return fail(ENKF_ERR_NOT_SUPPORTED, "local_init: too many problems");
  if (d->n_prob > 0 && (!win_start || !win_len || !state_idx))
    return fail(ENKF_ERR_INVALID_ARG, "local_init: window arrays are NULL");
  if (d->tune < ENKF_LOCAL_TUNE_DEFAULT || d->tune > ENKF_LOCAL_TUNE_PREFIX)
    return fail(ENKF_ERR_INVALID_ARG, "local_init: tune outside [0, 3]");
  for (int64_t p = 0; p < d->n_prob; ++p) {
    if (win_start[p] < 0 || win_start[p] >= d->n_glob || win_len[p] < 1 || win_len[p] > d->n_glob ||
        state_idx[p] < 0 || state_idx[p] >= d->n_state)
      return fail(ENKF_ERR_INVALID_ARG, "local_init: window " + std::to_string(p) + " out of range");
  }
  LocalPlan* pl = new (std::nothrow) LocalPlan();
  if (!pl) return fail(ENKF_ERR_OUT_OF_MEMORY, "local_init: plan");
  pl->desc = *d;
  pl->stream = static_cast<hipStream_t>(stream);
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      pl->n_cu = cus;
  }
  pl->max_blocks = pl->n_cu * 4;
  const int64_t P = d->n_prob;
  const size_t bytes = sizeof(int64_t) * 3 * (size_t)std::max<int64_t>(P, 1) +
                       sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(P, 1) +
                       sizeof(int32_t) * (size_t)(pl->max_blocks + 1) + 256 * 7;
  if (hipMalloc(&pl->ws, bytes) != hipSuccess) {
    pl->ws = nullptr;
    delete pl;
    return fail(ENKF_ERR_OUT_OF_MEMORY, "local_init: workspace");
  }
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = (off + b + 255) / 256 * 256; return o; };
  pl->win_start = reinterpret_cast<int64_t*>(pl->ws + take(sizeof(int64_t) * std::max<int64_t>(P, 1)));
  pl->win_len = reinterpret_cast<int64_t*>(pl->ws + take(sizeof(int64_t) * std::max<int64_t>(P, 1)));
  pl->state_idx = reinterpret_cast<int64_t*>(pl->ws + take(sizeof(int64_t) * std::max<int64_t>(P, 1)));
  pl->sched = reinterpret_cast<int32_t*>(pl->ws + take(sizeof(int32_t) * std::max<int64_t>(P, 1)));
  pl->sched_off = reinterpret_cast<int32_t*>(pl->ws + take(sizeof(int32_t) * (pl->max_blocks + 1)));
  pl->status = reinterpret_cast<unsigned*>(pl->ws + take(sizeof(unsigned) * 4));
  pl->psched = reinterpret_cast<int32_t*>(pl->ws + take(sizeof(int32_t) * std::max<int64_t>(P, 1)));
  hipStream_t s = pl->stream;
  enkf_status st = ENKF_SUCCESS;
  if (P > 0) {
    if (hipMemcpyAsync(pl->win_start, win_start, sizeof(int64_t) * P, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(pl->win_len, win_len, sizeof(int64_t) * P, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(pl->state_idx, state_idx, sizeof(int64_t) * P, hipMemcpyHostToDevice, s) != hipSuccess)
      st = fail(ENKF_ERR_HIP, "local_init: copies");
  }
  if (st == ENKF_SUCCESS && hipMemsetAsync(pl->status, 0, sizeof(unsigned) * 4, s) != hipSuccess)
    st = fail(ENKF_ERR_HIP, "local_init: status");
  pl->len_h.assign(win_len, win_len + P);
  if (st == ENKF_SUCCESS) st = pl->set_config(32, 2);
  int64_t rows = 0;                               // rows of all windows
  for (int64_t p = 0; p < P; ++p) rows += win_len[p];
  const bool want_prefix = d->tune == ENKF_LOCAL_TUNE_TIME || d->tune == ENKF_LOCAL_TUNE_PREFIX ||
                           (d->tune == ENKF_LOCAL_TUNE_DEFAULT && rows >= d->n_glob);
  if (st == ENKF_SUCCESS && P > 0 && want_prefix) st = pl->init_prefix(win_start, state_idx);
  if (st == ENKF_SUCCESS && d->tune == ENKF_LOCAL_TUNE_PREFIX && P > 0 && !pl->prefix_ok)
    st = fail(ENKF_ERR_NOT_SUPPORTED, "local_init: the prefix sums of this ring exceed their workspace limit");
  if (st != ENKF_SUCCESS) {
    delete pl;
    return st;
  }
  if (pl->prefix_ok && d->tune != ENKF_LOCAL_TUNE_TIME) pl->path = ENKF_LOCAL_PATH_PREFIX;
  pl->tuned = d->tune != ENKF_LOCAL_TUNE_TIME;
  *out = reinterpret_cast<enkf_local_plan>(pl);
  return ENKF_SUCCESS;
}

enkf_status enkf_local_analysis(enkf_local_plan plan, const double* r, const float* V, const float* D, int64_t ldv,
                                const float* XB, int64_t ldx, float* XA, int64_t ldxa, double* gamma) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "local_analysis: plan is NULL");
  LocalPlan* pl = reinterpret_cast<LocalPlan*>(plan);
  const enkf_local_desc& d = pl->desc;
  if (d.n_prob == 0) return ENKF_SUCCESS;
  if (!r || !V || !D || !XB || !XA) return fail(ENKF_ERR_INVALID_ARG, "local_analysis: NULL pointer");
  if (ldv < d.n_glob || ldx < d.n_state || ldxa < d.n_prob)
    return fail(ENKF_ERR_INVALID_ARG, "local_analysis: leading dimension too small");
  LocalArgs& a = pl->args;
  a.n_glob = d.n_glob;
  a.N = d.n_ens;
  a.ldv = ldv;
  a.ldx = ldx;
  a.ldxa = ldxa;
  a.n_prob = d.n_prob;
  a.r = r;
  a.V = V;
  a.D = D;
  a.XB = XB;
  a.XA = XA;
  a.gamma = gamma;
  a.win_start = pl->win_start;
  a.win_len = pl->win_len;
  a.state_idx = pl->state_idx;
  a.sched = pl->sched;
  a.sched_off = pl->sched_off;
  a.status = pl->status;
  a.inv_sqrt = 1.0 / std::sqrt((double)(d.n_ens - 1));
  // byte offset of the last element of V and D
  pl->o32 = (uint64_t)(d.n_glob - 1 + (int64_t)(d.n_ens - 1) * ldv) * 4u <= (uint64_t)UINT32_MAX;
  pl->pargs.ldv = ldv;
  pl->pargs.r = r;
  pl->pargs.V = V;
  pl->pargs.D = D;
  enkf_status st;
  if (!pl->tuned) {
    // time every configuration on this data and keep the fastest
    const int kcs[2] = {32, 64};
    const int bpcs[4] = {1, 2, 3, 4};
    float best = 1e30f;
    int best_kc = 32, best_bpc = 2, best_path = ENKF_LOCAL_PATH_STREAM;
    hipEvent_t e0, e1;
    ENKF_HIP_CHECK(hipEventCreate(&e0));
    ENKF_HIP_CHECK(hipEventCreate(&e1));
    for (int path : {ENKF_LOCAL_PATH_STREAM, ENKF_LOCAL_PATH_PREFIX})
      for (int kc : kcs)
      for (int bpc : bpcs) {
        if (path == ENKF_LOCAL_PATH_PREFIX && (!pl->prefix_ok || kc != kcs[0] || bpc != bpcs[0])) continue;
        pl->path = path;
        if (path == ENKF_LOCAL_PATH_STREAM) {
          st = pl->set_config(kc, bpc);
          if (st != ENKF_SUCCESS) return st;
        }
        st = pl->launch_direct();
        if (st != ENKF_SUCCESS) return st;
        float tmin = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          ENKF_HIP_CHECK(hipEventRecord(e0, pl->stream));
          st = pl->launch_direct();
          if (st != ENKF_SUCCESS) return st;
          ENKF_HIP_CHECK(hipEventRecord(e1, pl->stream));
          ENKF_HIP_CHECK(hipEventSynchronize(e1));
          float ms = 0.f;
          ENKF_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
          tmin = std::min(tmin, ms);
        }
        if (tmin < best) {
          best = tmin;
          best_kc = kc;
          best_bpc = bpc;
          best_path = path;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = pl->set_config(best_kc, best_bpc);
    if (st != ENKF_SUCCESS) return st;
    pl->path = best_path;
    pl->tuned = true;
  }
  if (!pl->exec || pl->graph_func != pl->main_func()) {
    st = pl->build_graph();
    if (st != ENKF_SUCCESS) return st;
  } else {
    st = pl->set_graph_params();
    if (st != ENKF_SUCCESS) return st;
  }
  ENKF_HIP_CHECK(hipGraphLaunch(pl->exec, pl->stream));
  return ENKF_SUCCESS;
}

enkf_status enkf_local_sync(enkf_local_plan plan, int32_t* rows_per_stage, int32_t* blocks) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "local_sync: plan is NULL");
  LocalPlan* pl = reinterpret_cast<LocalPlan*>(plan);
  ENKF_HIP_CHECK(hipStreamSynchronize(pl->stream));
  unsigned st = 0;
  ENKF_HIP_CHECK(hipMemcpy(&st, pl->status, sizeof(unsigned), hipMemcpyDeviceToHost));
  const bool pfx = pl->path == ENKF_LOCAL_PATH_PREFIX;
  if (rows_per_stage) *rows_per_stage = pfx ? 0 : pl->kc;
  if (blocks) *blocks = pfx ? (int32_t)pl->desc.n_prob : pl->nblocks;
  if (st != 0) return fail(static_cast<enkf_status>(st), "local_analysis: a pivot or r_i was not finite and > 0");
  return ENKF_SUCCESS;
}

enkf_status enkf_local_get_path(enkf_local_plan plan, int32_t* path) {
  if (!plan || !path) return fail(ENKF_ERR_INVALID_ARG, "local_get_path: NULL argument");
  *path = reinterpret_cast<LocalPlan*>(plan)->path;
  return ENKF_SUCCESS;
}

void enkf_local_destroy(enkf_local_plan plan) {
  if (!plan) return;
  delete reinterpret_cast<LocalPlan*>(plan);
}

}  // extern "C"
