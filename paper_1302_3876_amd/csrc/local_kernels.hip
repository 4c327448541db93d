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

  enkf_status set_config(int kc_, int blocks_per_cu);
  enkf_status launch_direct();
  enkf_status build_graph();
  ~LocalPlan();
};

LocalPlan::~LocalPlan() {
  if (stream || ws) (void)hipStreamSynchronize(stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ws) (void)hipFree(ws);
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

enkf_status LocalPlan::launch_direct() {
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
  void* kargs[] = {&args};
  kp.func = const_cast<void*>(kernel_for(kc, o32));
  graph_func = kp.func;
  kp.gridDim = dim3(nblocks);
  kp.blockDim = dim3(LT);
  kp.sharedMemBytes = 0;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  ENKF_HIP_CHECK(hipGraphAddKernelNode(&node, graph, nullptr, 0, &kp));
  ENKF_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
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
  const size_t bytes = sizeof(int64_t) * 3 * (size_t)std::max<int64_t>(P, 1) + sizeof(int32_t) * (size_t)std::max<int64_t>(P, 1) +
                       sizeof(int32_t) * (size_t)(pl->max_blocks + 1) + 256 * 6;
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
  if (st != ENKF_SUCCESS) {
    delete pl;
    return st;
  }
  pl->tuned = d->tune == 0;
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
  enkf_status st;
  if (!pl->tuned) {
    // time every configuration on this data and keep the fastest
    const int kcs[2] = {32, 64};
    const int bpcs[4] = {1, 2, 3, 4};
    float best = 1e30f;
    int best_kc = 32, best_bpc = 2;
    hipEvent_t e0, e1;
    ENKF_HIP_CHECK(hipEventCreate(&e0));
    ENKF_HIP_CHECK(hipEventCreate(&e1));
    for (int kc : kcs)
      for (int bpc : bpcs) {
        st = pl->set_config(kc, bpc);
        if (st != ENKF_SUCCESS) return st;
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
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = pl->set_config(best_kc, best_bpc);
    if (st != ENKF_SUCCESS) return st;
    pl->tuned = true;
  }
  if (!pl->exec || pl->graph_func != kernel_for(pl->kc, pl->o32)) {
    st = pl->build_graph();
    if (st != ENKF_SUCCESS) return st;
  } else {
    hipKernelNodeParams kp{};
    void* kargs[] = {&pl->args};
    kp.func = const_cast<void*>(kernel_for(pl->kc, pl->o32));
    kp.gridDim = dim3(pl->nblocks);
    kp.blockDim = dim3(LT);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    ENKF_HIP_CHECK(hipGraphExecKernelNodeSetParams(pl->exec, pl->node, &kp));
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
  if (rows_per_stage) *rows_per_stage = pl->kc;
  if (blocks) *blocks = pl->nblocks;
  if (st != 0) return fail(static_cast<enkf_status>(st), "local_analysis: a pivot or r_i was not finite and > 0");
  return ENKF_SUCCESS;
}

void enkf_local_destroy(enkf_local_plan plan) {
  if (!plan) return;
  delete reinterpret_cast<LocalPlan*>(plan);
}

}  // extern "C"
