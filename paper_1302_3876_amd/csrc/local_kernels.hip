// Batched localized analyses (enkf_local.h), gfx950.
//
// One launch runs every local problem. Blocks take statically scheduled
// lists of problems (longest window first, dealt to the least-loaded block).
// Per problem, 256 threads:
//  1. one streaming pass over the window's rows forms
//       [A | B] = Vs^T [Vs | Ds],  Vs = R^{-1/2} V_p, Ds = R^{-1/2} D_p,
//     on FP32 matrix cores (16x16x4); the FP32 accumulators are emptied
//     into FP64 after every stage of rows; waves 0-1 own A, waves 2-3 own B;
//  2. M = I + A = L D L^T in FP64 in LDS (right-looking); D holds the
//     pivots gamma_k of the iterative formula (Section 3.3);
//  3. y = M^{-1} delta with delta the centred ensemble row of the state
//     point (wave 0, forward and backward substitution with shuffles);
//  4. since V_p^T Z_p = M^{-1} B (the Woodbury form of eq. SWM with one
//     panel), the centre-point update is xa = x^B_s + (y^T B)/sqrt(N-1)
//     (Section 3.1), formed by waves 2-3 from their FP64 accumulators.
// The ensemble is padded to 64 members (zero anomalies give identity rows of
// M and zero products).
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
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

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int KC>
__global__ __launch_bounds__(LT) void local_kernel(LocalArgs a) {
  constexpr int LDK = KC + 1;
  __shared__ float Vt[LN * LDK];   // Vt[col][k] = V[g_k, col] / sqrt(r_{g_k})
  __shared__ float Dt[LN * LDK];
  __shared__ double M[LN * LDM];
  __shared__ double rs_s[KC];
  __shared__ double yv[LN];
  const int t = threadIdx.x, l = t % 64, w = t / 64;
  const int beg = a.sched_off[blockIdx.x], end = a.sched_off[blockIdx.x + 1];
  for (int q = beg; q < end; ++q) {
    const int p = a.sched[q];
    const int64_t g0 = a.win_start[p], m = a.win_len[p], s = a.state_idx[p];

    // 1. [A | B] over the window
    mf_f4 acc[4][2];
    double wide[4][2][4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        acc[ti][tj] = mf_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) wide[ti][tj][r] = 0.0;
      }
    for (int64_t i0 = 0; i0 < m; i0 += KC) {
      __syncthreads();
      if (t < KC) {
        const int64_t i = i0 + t;
        double v = 0.0;
        if (i < m) {
          int64_t g = g0 + i;
          if (g >= a.n_glob) g -= a.n_glob;
          const double rv = a.r[g];
          if (!(rv > 0.0) || !__builtin_isfinite(rv)) atomicOr(a.status, kStatusNotSpd);
          v = 1.0 / sqrt(rv);
        }
        rs_s[t] = v;
      }
      __syncthreads();
      for (int e = t; e < KC * LN; e += LT) {
        const int kk = e % KC, c = e / KC;
        const int64_t i = i0 + kk;
        float v = 0.f, d = 0.f;
        if (i < m && c < a.N) {
          int64_t g = g0 + i;
          if (g >= a.n_glob) g -= a.n_glob;
          const double sc = rs_s[kk];
          v = (float)((double)a.V[g + (int64_t)c * a.ldv] * sc);
          d = (float)((double)a.D[g + (int64_t)c * a.ldv] * sc);
        }
        Vt[c * LDK + kk] = v;
        Dt[c * LDK + kk] = d;
      }
      __syncthreads();
      const float* X = (w < 2) ? Vt : Dt;
      const int cbase = 32 * (w % 2);
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        float aop[4], bop[2];
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) aop[ti] = Vt[(16 * ti + l % 16) * LDK + kk + l / 16];
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) bop[tj] = X[(cbase + 16 * tj + l % 16) * LDK + kk + l / 16];
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj)
            acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[ti], bop[tj], acc[ti][tj], 0, 0, 0);
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
          for (int r = 0; r < 4; ++r) wide[ti][tj][r] += (double)acc[ti][tj][r];
          acc[ti][tj] = mf_f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
    // 2. M = I + A, then L D L^T
    if (w < 2) {
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti + 4 * (l / 16) + r;
            const int col = 32 * w + 16 * tj + l % 16;
            M[row * LDM + col] = wide[ti][tj][r] + (row == col ? 1.0 : 0.0);
          }
    }
    __syncthreads();
    for (int j = 0; j < LN; ++j) {
      const double d = M[j * LDM + j];
      const double inv_d = 1.0 / d;
      if (t == 0 && j < a.N) {
        if (a.gamma) a.gamma[p + (int64_t)j * a.n_prob] = d;
        if (!(d > 0.0) || !__builtin_isfinite(d)) atomicOr(a.status, kStatusNotSpd);
      }
      const int nr = LN - j - 1;
      for (int e = t; e < nr * nr; e += LT) {
        const int i = j + 1 + e / nr, k = j + 1 + e % nr;
        if (k <= i) M[i * LDM + k] -= M[i * LDM + j] * M[k * LDM + j] * inv_d;
      }
      __syncthreads();
      for (int i = j + 1 + t; i < LN; i += LT) M[i * LDM + j] *= inv_d;
      __syncthreads();
    }
    // 3. y = M^{-1} delta (wave 0)
    if (w == 0) {
      const double x = (l < a.N) ? (double)a.XB[s + (int64_t)l * a.ldx] : 0.0;
      const double mean = wsum(x) / (double)a.N;
      double z = (l < a.N) ? x - mean : 0.0;
      for (int k = 0; k < LN; ++k) {
        const double zk = __shfl(z, k, 64);
        if (l > k) z -= M[l * LDM + k] * zk;
      }
      z = z / M[l * LDM + l];
      for (int k = LN - 1; k >= 0; --k) {
        const double yk = __shfl(z, k, 64);
        if (l < k) z -= M[k * LDM + l] * yk;
      }
      yv[l] = z;
    }
    __syncthreads();
    // 4. xa = x^B_s + (y^T B) / sqrt(N-1) (waves 2-3 hold B)
    if (w >= 2) {
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        double part = 0.0;
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) part += yv[16 * ti + 4 * (l / 16) + r] * wide[ti][tj][r];
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        const int col = 32 * (w - 2) + 16 * tj + l;
        if (l < 16 && col < a.N)
          a.XA[p + (int64_t)col * a.ldxa] = (float)((double)a.XB[s + (int64_t)col * a.ldx] + part * a.inv_sqrt);
      }
    }
  }
}

const void* kernel_for(int kc) {
  return kc == 64 ? reinterpret_cast<const void*>(&local_kernel<64>) : reinterpret_cast<const void*>(&local_kernel<32>);
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
  int nblocks = 0;
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
    heap.push({top.first + len_h[pidx] + 2 * LN, top.second});
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
  if (kc == 64) local_kernel<64><<<nblocks, LT, 0, stream>>>(args);
  else local_kernel<32><<<nblocks, LT, 0, stream>>>(args);
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
  kp.func = const_cast<void*>(kernel_for(kc));
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
  if (!pl->exec) {
    st = pl->build_graph();
    if (st != ENKF_SUCCESS) return st;
  } else {
    hipKernelNodeParams kp{};
    void* kargs[] = {&pl->args};
    kp.func = const_cast<void*>(kernel_for(pl->kc));
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
