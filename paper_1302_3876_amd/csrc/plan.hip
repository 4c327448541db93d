// Plan: workspace layout and the launch sequences of the factorisation,
// solve and analysis, for the plain, blocked and mixed-precision forms.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "diag.h"
#include "gemm_lowp.h"
#include "gemm_mfma.h"
#include "panel.h"
#include "plan.h"

namespace enkf {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool vec_ok(const void* p, int64_t ld, int vw, size_t es) {
  return p == nullptr || (((uintptr_t)p % (vw * es)) == 0 && (ld % vw) == 0);
}

__global__ void clear_words_kernel(unsigned* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

// Byte and flop model of one plain sweep launch over m columns of n rows:
// read and write the m columns, read u_k and v_{k+1} (Step 1: the source
// columns and r instead of u_k); flops 4 m n (update + look-ahead product).
void sweep_model(int64_t n, int m, size_t es, bool step1, bool look, double* by, double* fl) {
  const double cols = 2.0 * m + (look ? 1.0 : 0.0) + (step1 ? 0.0 : 1.0);
  *by = cols * (double)n * (double)es + (step1 ? 8.0 * (double)n : 0.0);
  *fl = (double)n * m * (look ? 4.0 : 2.0);
}

}  // namespace

// Last-level (infinity) cache of the MI355X: 256 MiB.
constexpr double kMallBytes = 256.0 * 1024.0 * 1024.0;

const void* Plan::vcol(int k) const { return static_cast<const char*>(V) + (size_t)k * (size_t)ldv * es; }

// Panel products in the working type; narrow math types round the FP32
// operands when they are staged.
enkf_status Plan::panel_tn(int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb, double* Gout,
                           int64_t ldg) {
  if (mixed && desc.math != ENKF_MATH_F32)
    return launch_tn_lowp(desc.math, n, a, m, static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb,
                          Gout, ldg, tn_part, stream);
  return launch_tn(wdt, n, a, m, A, lda, B, ldb, Gout, ldg, tn_part, stream);
}

enkf_status Plan::panel_nn(const NnArgs& a) {
  if (mixed && desc.math != ENKF_MATH_F32) return launch_nn_lowp(desc.math, NN_UPDATE, a, stream);
  return launch_nn(wdt, NN_UPDATE, a, stream);
}

enkf_status Plan::create(const enkf_sm_desc& d, const double* r_, const void* V_, int64_t ldv_, hipStream_t s,
                         char* ext_ws, size_t ext_bytes) {
  desc = d;
  r = r_;
  V = V_;
  ldv = ldv_;
  stream = s;
  es = dtype_size(d.dtype);
  max_nrhs = d.max_nrhs > 0 ? d.max_nrhs : d.n_ens;
  pivot = (d.flags & ENKF_FLAG_PIVOT) != 0;
  const int64_t n = d.n_obs;
  const int N = d.n_ens;
  const int mcols = std::max(N, max_nrhs);
  const bool blocked = d.algo == ENKF_SM_BLOCKED;
  mixed = blocked && d.dtype == ENKF_F64 && d.math != ENKF_MATH_F64;
  // FP64 panels with FP64 refinement: the Woodbury panel update is not
  // backward stable, a few residual corrections restore the level formula's
  // accuracy on ill-conditioned systems
  refine64 = blocked && d.dtype == ENKF_F64 && d.math == ENKF_MATH_F64 && d.refine_max_iter > 0;
  // diagnostics need an FP64 V for the residual and a diagonal R (diag_factor
  // and diag_solve skip a plan with a block-diagonal R)
  diagnose = (d.flags & ENKF_FLAG_DIAGNOSE) != 0 && d.dtype == ENKF_F64 && N <= wnorm_max_n_ens();
  wdt = mixed ? ENKF_F32 : d.dtype;
  const size_t wes = dtype_size(wdt);
  autotune = blocked && d.block == 0 && (d.flags & ENKF_FLAG_AUTOTUNE) != 0;
  std::vector<int> widths;      // every panel width the workspace must serve
  if (blocked) {
    block = d.block > 0 ? d.block : std::min(N, kMaxPanel);
    if (block > kMaxPanel) return fail(ENKF_ERR_NOT_SUPPORTED, "init: panel width above 128");
    npanel = (N + block - 1) / block;
    if (d.dtype == ENKF_F32 && d.math != ENKF_MATH_F32)
      return fail(ENKF_ERR_NOT_SUPPORTED, "init: FP32 storage takes FP32 panels (narrower panels refine an FP64 solve)");
    widths = autotune ? tune_candidates(N) : std::vector<int>{block};
  }
  ldu = (int64_t)align_up((size_t)n, 64);

  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  // plain: U is followed by max_nrhs columns that hold Z during a fused
  // factorisation + solve, so one launch per level covers [U_{>k}, Z]
  const size_t oU = take((size_t)ldu * (N + (blocked ? 0 : max_nrhs)) * wes);
  const size_t oGamma = take(sizeof(double) * N);
  const size_t oStat = take(sizeof(unsigned) * 4);
  const size_t oG = take(sizeof(double) * (size_t)N * mcols);
  // split-K partials: the largest over every (a, m) product this plan runs
  int64_t tnp = tn_partial_elems(n, N, N);   // analysis V^T Z
  size_t sfac_elems = 0, pbuf_elems = 0, qbuf_elems = 0;
  for (const int b : widths) {
    const int np = (N + b - 1) / b;
    for (int p = 0; p < np; ++p) {
      const int k0 = p * b, bl = std::min(b, N - k0);
      tnp = std::max(tnp, tn_partial_elems(n, bl, N - k0));
      for (int m = 1; m <= max_nrhs; ++m) tnp = std::max(tnp, tn_partial_elems(n, bl, m));
    }
    sfac_elems = std::max(sfac_elems, (size_t)np * b * b);
    pbuf_elems = std::max(pbuf_elems, (size_t)b * (N + mcols));
    qbuf_elems = std::max(qbuf_elems, (size_t)b * mcols);
  }
  if (mixed || refine64 || diagnose)
    for (int m = 1; m <= max_nrhs; ++m) tnp = std::max(tnp, tn_partial_elems(n, N, m));
  const size_t oTn = take(sizeof(double) * (size_t)tnp);
  // right factor of an nn product, converted: inner dimension <= N, columns <= mcols
  const size_t oBt = take(nn_bt_bytes(N, mcols));
  size_t oP0 = 0, oP1 = 0, oSfac = 0, oPbuf = 0, oQbuf = 0, oVw = 0, oZw = 0, oRho = 0, oNorm = 0, oResPart = 0;
  size_t oGc = 0, oCb = 0, oPerm = 0, oRem = 0, oAct = 0;
  if (!blocked) {
    const size_t part_elems = (size_t)level_row_blocks(d.dtype, 1, n) * (N + max_nrhs);
    oP0 = take(sizeof(double) * part_elems);
    oP1 = take(sizeof(double) * part_elems);
    if (pivot) {
      oGc = take(sizeof(double) * N);
      oCb = take(sizeof(double) * N);
      oPerm = take(sizeof(int32_t) * N);
      oRem = take(sizeof(int32_t) * 2 * (size_t)N);
      oAct = take(sizeof(int32_t) * 2 * (size_t)(N + max_nrhs));
    }
  } else {
    oSfac = take(sizeof(double) * sfac_elems);
    oPbuf = take(sizeof(double) * pbuf_elems);
    oQbuf = take(sizeof(double) * qbuf_elems);
  }
  if (mixed) {
    oVw = take((size_t)ldu * N * sizeof(float));
    oZw = take((size_t)ldu * mcols * sizeof(float));
  }
  if (mixed || refine64 || diagnose) {
    oRho = take((size_t)ldu * mcols * sizeof(double));
    oNorm = take(sizeof(double) * (kNrmPart + (size_t)std::max(norm_partial_elems(), wnorm_partial_elems())));
    res_part_cap = nn_residual_part_elems(n, mcols);
    oResPart = take(sizeof(double) * (size_t)res_part_cap);
  }
  ws_bytes = off;
  if (ext_ws) {
    // the caller's workspace (the static scratch of the allocation-free call)
    if (ws_bytes > ext_bytes)
      return fail(ENKF_ERR_NOT_SUPPORTED, "workspace of " + std::to_string(ws_bytes) + " bytes exceeds the " +
                                              std::to_string(ext_bytes) + "-byte static scratch");
    ws = ext_ws;
    owns_ws = false;
  } else {
    hipError_t e = hipMalloc(&ws, ws_bytes);
    if (e != hipSuccess) {
      ws = nullptr;
      return fail(ENKF_ERR_OUT_OF_MEMORY, "init: workspace of " + std::to_string(ws_bytes) + " bytes");
    }
    owns_ws = true;
  }
  U = ws + oU;
  gamma = reinterpret_cast<double*>(ws + oGamma);
  status = reinterpret_cast<unsigned*>(ws + oStat);
  G = reinterpret_cast<double*>(ws + oG);
  tn_part = reinterpret_cast<double*>(ws + oTn);
  Bt = ws + oBt;
  if (!blocked) {
    part[0] = reinterpret_cast<double*>(ws + oP0);
    part[1] = reinterpret_cast<double*>(ws + oP1);
    if (pivot) {
      gcur = reinterpret_cast<double*>(ws + oGc);
      cbuf = reinterpret_cast<double*>(ws + oCb);
      perm = reinterpret_cast<int32_t*>(ws + oPerm);
      rem[0] = reinterpret_cast<int32_t*>(ws + oRem);
      rem[1] = rem[0] + N;
      act[0] = reinterpret_cast<int32_t*>(ws + oAct);
      act[1] = act[0] + N + max_nrhs;
    }
  } else {
    Sfac = reinterpret_cast<double*>(ws + oSfac);
    Pbuf = reinterpret_cast<double*>(ws + oPbuf);
    Qbuf = reinterpret_cast<double*>(ws + oQbuf);
  }
  if (mixed) {
    Vw = ws + oVw;
    Zw = ws + oZw;
  }
  if (mixed || refine64 || diagnose) {
    rho = reinterpret_cast<double*>(ws + oRho);
    norms = reinterpret_cast<double*>(ws + oNorm);
    res_part = reinterpret_cast<double*>(ws + oResPart);
  }
  // the status words start at zero (a fill kernel: valid under stream capture)
  clear_words_kernel<<<1, 64, 0, stream>>>(status, 4);
  ENKF_HIP_CHECK(hipGetLastError());
  last.rel_residual = -1.0;
  last.backward_error = -1.0;
  return ENKF_SUCCESS;
}

Plan::~Plan() {
  // a plan on a borrowed workspace neither waits nor frees: its kernels
  // reference no host state of the plan
  if (!owns_ws && !bws) return;
  if (stream || ws || bws) (void)hipStreamSynchronize(stream);
  if (ws && owns_ws) (void)hipFree(ws);
  if (bws) (void)hipFree(bws);
}

// Block-diagonal R: keep the block structure on the device and factor the
// blocks (Section 2.1). Offsets are validated by the caller.
enkf_status Plan::set_block_r(int64_t nb_, const int64_t* off_host) {
  block_r = true;
  nblk = nb_;
  max_bs = 0;
  std::vector<int64_t> poff_h(nblk + 1, 0);
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t sz = off_host[b + 1] - off_host[b];
    max_bs = std::max<int>(max_bs, (int)sz);
    poff_h[b + 1] = poff_h[b] + sz * sz;
  }
  const size_t bytes = sizeof(int64_t) * 2 * (size_t)(nblk + 1) + sizeof(double) * (size_t)poff_h[nblk];
  hipError_t e = hipMalloc(&bws, bytes);
  if (e != hipSuccess) {
    bws = nullptr;
    return fail(ENKF_ERR_OUT_OF_MEMORY, "init: block R workspace");
  }
  boff = reinterpret_cast<int64_t*>(bws);
  bpoff = boff + nblk + 1;
  Lf = reinterpret_cast<double*>(bpoff + nblk + 1);
  ENKF_HIP_CHECK(hipMemcpyAsync(boff, off_host, sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipMemcpyAsync(bpoff, poff_h.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice, stream));
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));   // poff_h leaves scope
  return ENKF_SUCCESS;
}

enkf_status Plan::factor_block_r(const double* Rblocks) {
  return launch_block_chol(nblk, boff, bpoff, Rblocks, Lf, status, stream);
}

// Step 1 of a block-R plan: Y = R^{-1} X in the working type.
enkf_status Plan::block_step1(enkf_dtype dt, int m, const void* X, int64_t ldx, void* Y, int64_t ldy) {
  TimedLaunch tl(&timing, stream, KC_STEP1, 2.0 * (double)desc.n_obs * m * dtype_size(dt),
                 2.0 * (double)desc.n_obs * m * max_bs);
  return launch_block_solve(dt, max_bs, nblk, m, boff, bpoff, Lf, X, ldx, Y, ldy, stream);
}

// ------------------------------------------------------------------ panel width
std::vector<int> tune_candidates(int N) {
  std::vector<int> c;
  for (const int b : {32, 64, 96, 128})
    if (b <= N) c.push_back(b);
  if (c.empty()) c.push_back(N);
  return c;
}

namespace {
struct TuneKey {
  int64_t n;
  int N, dtype, math, nrhs, block_r;
  bool operator<(const TuneKey& o) const {
    return std::tie(n, N, dtype, math, nrhs, block_r) < std::tie(o.n, o.N, o.dtype, o.math, o.nrhs, o.block_r);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;   // panel width picked per shape, for the life of the process
}  // namespace

// ENKF_FLAG_AUTOTUNE: time the factorisation and one solve of min(N,
// max_nrhs) right-hand sides (the columns of V, without refinement) for each
// candidate width on this plan's own data, and keep the fastest. A shape
// tuned before in this process reuses its width.
enkf_status Plan::tune_block() {
  if (!autotune) return ENKF_SUCCESS;
  const TuneKey key{desc.n_obs, desc.n_ens, (int)desc.dtype, (int)desc.math, max_nrhs, block_r ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      block = it->second;
      npanel = (desc.n_ens + block - 1) / block;
      return ENKF_SUCCESS;
    }
  }
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  const int nr = std::min(N, max_nrhs);
  const std::vector<int> cand = tune_candidates(N);
  void* scratch = nullptr;
  if (!mixed) {
    if (hipMalloc(&scratch, (size_t)ldu * nr * dtype_size(wdt)) != hipSuccess)
      return fail(ENKF_ERR_OUT_OF_MEMORY, "autotune: right-hand side scratch");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  enkf_status st = ENKF_SUCCESS;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(ENKF_ERR_HIP, "autotune: events");
  ntune = 0;
  int best = cand[0];
  float best_ms = 0.f;
  for (size_t ci = 0; ci < cand.size() && st == ENKF_SUCCESS; ++ci) {
    block = cand[ci];
    npanel = (N + block - 1) / block;
    float tmin = 0.f;
    for (int rep = 0; rep < 3 && st == ENKF_SUCCESS; ++rep) {   // rep 0 warms up
      if (mixed) st = launch_convert(n, nr, static_cast<const double*>(V), ldv, static_cast<float*>(Zw), ldu, nullptr,
                                     r, status, stream);
      if (st != ENKF_SUCCESS) break;
      if (hipEventRecord(e0, stream) != hipSuccess) { st = fail(ENKF_ERR_HIP, "autotune: event record"); break; }
      st = factor_blocked();
      if (st == ENKF_SUCCESS)
        st = mixed ? solve_blocked(nr, Zw, ldu, Zw, ldu, true) : solve_blocked(nr, V, ldv, scratch, ldu);
      if (st != ENKF_SUCCESS) break;
      float ms = 0.f;
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(ENKF_ERR_HIP, "autotune: event timing");
        break;
      }
      if (rep == 1 || (rep > 1 && ms < tmin)) tmin = ms;
    }
    if (st != ENKF_SUCCESS) break;
    if (ntune < kMaxTune) {
      tune_b[ntune] = cand[ci];
      tune_ms[ntune] = tmin;
      ++ntune;
    }
    if (ci == 0 || tmin < best_ms) {
      best = cand[ci];
      best_ms = tmin;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (scratch) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(scratch);
  }
  if (st != ENKF_SUCCESS) return st;
  block = best;
  npanel = (N + block - 1) / block;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = block;
  }
  // the trial factorisations may have latched a status; the real one
  // that follows latches it again
  return clear_status();
}

enkf_status Plan::factor() {
  enkf_status st = desc.algo == ENKF_SM_PLAIN ? factor_plain() : factor_blocked();
  if (st != ENKF_SUCCESS) return st;
  return diag_factor();
}

// ------------------------------------------------------------------ diagnostics
enkf_status Plan::diag_factor() {
  if (!diagnose || block_r) return ENKF_SUCCESS;
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  enkf_status st = launch_tn(ENKF_F64, n, N, N, V, ldv, V, ldv, G, N, tn_part, stream);
  if (st != ENKF_SUCCESS) return st;
  return launch_wnorm_estimate(n, N, r, G, N, norms + kNrmPart, norms + kNrmW, stream);
}

// After a synchronous solve: the FP64 residual of Z unless the form left
// it (plain and unrefined blocked solves; not possible when Z overwrote D),
// ||Z||^2, and eta = ||rho|| / (||W||_2 ||Z|| + ||D||) into `last`.
enkf_status Plan::diag_solve(int nrhs, const void* D, int64_t ldd, const void* Z, int64_t ldz) {
  last.backward_error = -1.0;
  if (!diagnose || block_r || nrhs == 0) return ENKF_SUCCESS;
  enkf_status st;
  if (!(mixed || refine64)) {
    const uintptr_t d0 = (uintptr_t)D, d1 = d0 + ((size_t)ldd * (nrhs - 1) + desc.n_obs) * es;
    const uintptr_t z0 = (uintptr_t)Z, z1 = z0 + ((size_t)ldz * (nrhs - 1) + desc.n_obs) * es;
    if (z0 < d1 && d0 < z1) return ENKF_SUCCESS;
    st = residual64(nrhs, D, ldd, Z, ldz, true);
    if (st != ENKF_SUCCESS) return st;
  }
  st = launch_sumsq(desc.n_obs, nrhs, static_cast<const double*>(Z), ldz, nullptr, norms + kNrmPart, norms + kNrmZ,
                    stream);
  if (st != ENKF_SUCCESS) return st;
  double h[kNrmW + 1];
  ENKF_HIP_CHECK(hipMemcpyAsync(h, norms, sizeof(h), hipMemcpyDeviceToHost, stream));
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  const double rn = std::sqrt(h[kNrmRho]), dn = std::sqrt(h[kNrmD]), zn = std::sqrt(h[kNrmZ]);
  last.rel_residual = dn > 0.0 ? rn / dn : rn;
  const double den = h[kNrmW] * zn + dn;
  last.backward_error = den > 0.0 ? rn / den : rn;
  return ENKF_SUCCESS;
}

// ------------------------------------------------------------------ plain
enkf_status Plan::factor_plain() {
  if (pivot) return sweep_pivot(0, nullptr, 0, nullptr, 0);
  if (small_plain(0)) return small_sweep(0, nullptr, 0, nullptr, 0, false);
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  const int w = level_vw(desc.dtype);
  const int vw = (n % w == 0 && vec_ok(U, ldu, w, es) && vec_ok(V, ldv, w, es)) ? w : 1;
  const int nb = level_row_blocks(desc.dtype, vw, n);
  // Step 1 for V: U0 = R^{-1} V and the products v_1^T u_j^{(0)} (block R:
  // the block solves first, then the same pass with no scaling).
  if (block_r) {
    enkf_status st = block_step1(desc.dtype, N, V, ldv, U, ldu);
    if (st != ENKF_SUCCESS) return st;
  }
  LevelArgs a{};
  a.n = n;
  a.vw = vw;
  a.status = status;
  a.X = U;
  a.ldx = ldu;
  a.m = N;
  a.src = block_r ? U : V;
  a.lds = block_r ? ldu : ldv;
  a.r = r;
  a.vnext = vcol(0);
  a.part_out = part[0];
  {
    double by, fl;
    sweep_model(n, N, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_STEP1, by, fl);
    enkf_status st = launch_level(desc.dtype, a, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  // Level k (0-based, k < N-1) forms gamma_k and updates U columns k+1..N-1.
  for (int k = 0; k + 1 < N; ++k) {
    LevelArgs b{};
    b.n = n;
    b.vw = vw;
    b.status = status;
    b.X = static_cast<char*>(U) + (size_t)(k + 1) * ldu * es;
    b.ldx = ldu;
    b.m = N - k - 1;
    b.uk = static_cast<char*>(U) + (size_t)k * ldu * es;
    b.gamma_out = gamma + k;
    b.prev = part[k & 1];
    b.prev_m = N - k;
    b.prev_off = 1;
    b.vnext = vcol(k + 1);
    b.part_out = part[(k + 1) & 1];
    double by, fl;
    sweep_model(n, b.m, es, false, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_INIT_SWEEP, by, fl);
    enkf_status st = launch_level(desc.dtype, b, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  // The last pivot has no U columns left to update.
  return launch_gamma_from_partials(part[(N - 1) & 1], nb, 0, gamma + (N - 1), status, stream);
}

enkf_status Plan::solve_plain(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  if (nrhs == 0) return ENKF_SUCCESS;
  if (small_plain(nrhs) && small_plain(0)) return small_sweep(nrhs, D, ldd, Z, ldz, true);
  const int w = level_vw(desc.dtype);
  const int vw = (n % w == 0 && vec_ok(U, ldu, w, es) && vec_ok(V, ldv, w, es) && vec_ok(D, ldd, w, es) &&
                  vec_ok(Z, ldz, w, es)) ? w : 1;
  if (block_r) {
    enkf_status st = block_step1(desc.dtype, nrhs, D, ldd, Z, ldz);
    if (st != ENKF_SUCCESS) return st;
  }
  LevelArgs a{};
  a.n = n;
  a.vw = vw;
  a.status = status;
  a.X = Z;
  a.ldx = ldz;
  a.m = nrhs;
  a.src = block_r ? Z : D;
  a.lds = block_r ? ldz : ldd;
  a.r = r;
  a.vnext = vcol(0);
  if (pivot) {
    a.vnext = V;
    a.vn_idx = perm;
    a.ldv_idx = ldv;
  }
  a.part_out = part[0];
  {
    double by, fl;
    sweep_model(n, nrhs, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_STEP1, by, fl);
    enkf_status st = launch_level(desc.dtype, a, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  for (int k = 0; k < N; ++k) {
    LevelArgs b{};
    b.n = n;
    b.vw = vw;
    b.status = status;
    b.X = Z;
    b.ldx = ldz;
    b.m = nrhs;
    b.uk = static_cast<char*>(U) + (size_t)k * ldu * es;
    b.gamma_in = gamma + k;
    b.prev = part[k & 1];
    b.prev_m = nrhs;
    b.prev_off = 0;
    b.vnext = (k + 1 < N) ? vcol(k + 1) : nullptr;
    if (pivot) {
      b.uk = U;
      b.uk_idx = perm + k;
      b.ldu_idx = ldu;
      if (k + 1 < N) {
        b.vnext = V;
        b.vn_idx = perm + k + 1;
        b.ldv_idx = ldv;
      }
    }
    b.part_out = part[(k + 1) & 1];
    double by, fl;
    sweep_model(n, nrhs, es, false, b.vnext != nullptr, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_SOLVE_SWEEP, by, fl);
    enkf_status st = launch_level(desc.dtype, b, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  return ENKF_SUCCESS;
}

// Factorisation and solve in one level loop (Section 3.3): Step 1 for V and
// for D, then per level k one launch over [U columns k+1..N-1, Z] that forms
// gamma_k, applies h_k to every active column and leaves the products with
// v_{k+1}. Z lives in the columns after U during the loop; the last level
// writes it to the caller's buffer. Leaves the same factor as factor_plain.
// A small FP64 system (no pivoting, diagonal R): the factorisation (nrhs =
// 0), the fused factorisation + solve, or a solve with the stored factor, in
// one launch of small_sweep_kernel.
bool Plan::small_plain(int nrhs) const {
  return desc.dtype == ENKF_F64 && !pivot && !block_r && desc.n_obs <= kSmallSweepMaxRows &&
         small_sweep_lds_bytes(desc.n_obs, desc.n_ens, nrhs) <= kSmallSweepMaxLds;
}

enkf_status Plan::small_sweep(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool solve_only) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  SmallSweepArgs a{};
  a.n = n;
  a.N = N;
  a.nrhs = nrhs;
  a.r = r;
  a.V = static_cast<const double*>(V);
  a.ldv = ldv;
  a.D = static_cast<const double*>(D);
  a.ldd = ldd;
  a.U = static_cast<double*>(U);
  a.ldu = ldu;
  a.Uin = solve_only ? static_cast<const double*>(U) : nullptr;
  a.Z = static_cast<double*>(Z);
  a.ldz = ldz;
  a.gamma = gamma;
  a.status = status;
  const double cols = solve_only ? nrhs : N + nrhs;
  TimedLaunch tl(&timing, stream, solve_only ? KC_SOLVE_SWEEP : (nrhs ? KC_FUSED_SWEEP : KC_INIT_SWEEP),
                 8.0 * n * (2.0 * cols + N + (solve_only ? N : 0)) + 8.0 * n, 4.0 * n * N * cols);
  return launch_small_sweep(a, stream);
}

enkf_status Plan::factor_solve_plain(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  if (nrhs == 0) return factor_plain();
  if (pivot) return sweep_pivot(nrhs, D, ldd, Z, ldz);
  if (small_plain(nrhs)) return small_sweep(nrhs, D, ldd, Z, ldz, false);
  if (small_plain(0)) {
    // the factor fits the single-block path but [U, Z] does not: factor
    // there and solve with the level launches, as refactor + solve would
    enkf_status st = factor_plain();
    return st != ENKF_SUCCESS ? st : solve_plain(nrhs, D, ldd, Z, ldz);
  }
  // One loop over [U, Z] saves a launch per level, but its per-level working
  // set, (N - k + nrhs) columns, can exceed the 256 MiB last-level (MALL)
  // cache, while the separate U and Z loops each stay inside it when their
  // own columns fit: then the two loops move fewer bytes from HBM.
  const double fused_bytes = (double)(N + nrhs) * (double)n * (double)es;
  const double split_bytes = (double)std::max(N, nrhs) * (double)n * (double)es;
  const bool split = fused_bytes > kMallBytes && split_bytes <= kMallBytes;
  if (block_r || split) {
    enkf_status st = factor_plain();
    return st != ENKF_SUCCESS ? st : solve_plain(nrhs, D, ldd, Z, ldz);
  }
  const int w = level_vw(desc.dtype);
  const int vw = (n % w == 0 && vec_ok(U, ldu, w, es) && vec_ok(V, ldv, w, es) && vec_ok(D, ldd, w, es) &&
                  vec_ok(Z, ldz, w, es)) ? w : 1;
  const int nb = level_row_blocks(desc.dtype, vw, n);
  char* Ub = static_cast<char*>(U);
  void* Zb = Ub + (size_t)N * ldu * es;
  for (int half = 0; half < 2; ++half) {
    LevelArgs a{};
    a.n = n;
    a.vw = vw;
    a.status = status;
    a.X = half == 0 ? U : Zb;
    a.ldx = ldu;
    a.m = half == 0 ? N : nrhs;
    a.src = half == 0 ? V : D;
    a.lds = half == 0 ? ldv : ldd;
    a.r = r;
    a.vnext = vcol(0);
    a.part_out = part[0] + (half == 0 ? 0 : (size_t)N * nb);
    double by, fl;
    sweep_model(n, a.m, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_STEP1, by, fl);
    enkf_status st = launch_level(desc.dtype, a, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  for (int k = 0; k < N; ++k) {
    LevelArgs b{};
    b.n = n;
    b.vw = vw;
    b.status = status;
    b.X = Ub + (size_t)(k + 1) * ldu * es;
    b.ldx = ldu;
    b.m = N - k - 1 + nrhs;
    b.uk = Ub + (size_t)k * ldu * es;
    b.gamma_out = gamma + k;
    b.prev = part[k & 1];
    b.prev_m = N - k + nrhs;
    b.prev_off = 1;
    b.vnext = (k + 1 < N) ? vcol(k + 1) : nullptr;
    b.part_out = part[(k + 1) & 1];
    if (k + 1 == N) {
      b.dst = Z;
      b.ldo = ldz;
    }
    double by, fl;
    sweep_model(n, b.m, es, false, b.vnext != nullptr, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_FUSED_SWEEP, by, fl);
    enkf_status st = launch_level(desc.dtype, b, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  return ENKF_SUCCESS;
}

// Plain sweeps with the pivoting of Section 3.4 (factorisation, and the Z
// columns too when nrhs > 0). U keeps V's column order (column j of U holds
// u_j); perm[k] is the column used at level k and every level's active list
// is built on the device by the pivot kernel, which also forms gamma_k, so
// the host never waits. Z lives in the columns after U during the loop and
// is copied to the caller's buffer at the end.
enkf_status Plan::sweep_pivot(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  const int w = level_vw(desc.dtype);
  bool ok = n % w == 0 && vec_ok(U, ldu, w, es) && vec_ok(V, ldv, w, es);
  if (nrhs > 0) ok = ok && vec_ok(D, ldd, w, es) && vec_ok(Z, ldz, w, es);
  const int vw = ok ? w : 1;
  const int nb = level_row_blocks(desc.dtype, vw, n);
  char* Ub = static_cast<char*>(U);
  void* Zb = Ub + (size_t)N * ldu * es;
  enkf_status st;
  {
    // candidates 1 + v_i^T R^{-1} v_i and the first pivot
    TimedLaunch tl(&timing, stream, KC_STEP1, (double)N * n * es + 8.0 * n, 3.0 * (double)N * n);
    st = launch_diag_partials(desc.dtype, n, N, V, ldv, r, nb, part[1], stream);
    if (st != ENKF_SUCCESS) return st;
    PivotArgs pa{};
    pa.init = 1;
    pa.N = N;
    pa.part = part[1];
    pa.nb = nb;
    pa.perm = perm;
    pa.gcur = gcur;
    pa.rem_out = rem[0];
    pa.status = status;
    st = launch_pivot(pa, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  for (int half = 0; half < (nrhs > 0 ? 2 : 1); ++half) {
    LevelArgs a{};
    a.n = n;
    a.vw = vw;
    a.status = status;
    a.X = half == 0 ? U : Zb;
    a.ldx = ldu;
    a.m = half == 0 ? N : nrhs;
    a.src = half == 0 ? V : D;
    a.lds = half == 0 ? ldv : ldd;
    a.r = r;
    a.vnext = V;
    a.vn_idx = perm;
    a.ldv_idx = ldv;
    a.part_out = part[0] + (half == 0 ? 0 : (size_t)N * nb);
    double by, fl;
    sweep_model(n, a.m, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_STEP1, by, fl);
    st = launch_level(desc.dtype, a, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  const int cls = nrhs > 0 ? KC_FUSED_SWEEP : KC_INIT_SWEEP;
  for (int k = 0; k < N; ++k) {
    const int m = N - k - 1 + nrhs;
    double by, fl;
    sweep_model(n, m, es, false, k + 1 < N, &by, &fl);
    TimedLaunch tl(&timing, stream, cls, by, fl);
    PivotArgs pa{};
    pa.k = k;
    pa.N = N;
    pa.nz = nrhs;
    pa.part = part[k & 1];
    pa.nb = nb;
    pa.perm = perm;
    pa.gamma = gamma;
    pa.gcur = gcur;
    pa.cbuf = cbuf;
    pa.rem_in = rem[k & 1];
    pa.rem_out = rem[(k + 1) & 1];
    pa.act_out = act[k & 1];
    pa.status = status;
    st = launch_pivot(pa, stream);
    if (st != ENKF_SUCCESS) return st;
    if (m == 0) continue;
    LevelArgs b{};
    b.n = n;
    b.vw = vw;
    b.status = status;
    b.X = U;
    b.ldx = ldu;
    b.m = m;
    b.colmap = act[k & 1];
    b.uk = U;
    b.uk_idx = perm + k;
    b.ldu_idx = ldu;
    b.gamma_in = gamma + k;
    b.prev = part[k & 1];
    b.prev_m = N - k + nrhs;
    if (k + 1 < N) {
      b.vnext = V;
      b.vn_idx = perm + k + 1;
      b.ldv_idx = ldv;
    }
    b.part_out = part[(k + 1) & 1];
    st = launch_level(desc.dtype, b, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  if (nrhs > 0)
    ENKF_HIP_CHECK(hipMemcpy2DAsync(Z, (size_t)ldz * es, Zb, (size_t)ldu * es, (size_t)n * es, nrhs,
                                    hipMemcpyDeviceToDevice, stream));
  return ENKF_SUCCESS;
}

enkf_status Plan::factor_solve(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info) {
  if (desc.algo != ENKF_SM_PLAIN) {
    enkf_status st = factor();
    if (st != ENKF_SUCCESS) return st;
    return solve(nrhs, D, ldd, Z, ldz, info);
  }
  enkf_status st = factor_solve_plain(nrhs, D, ldd, Z, ldz);
  last.refine_iters = 0;
  last.rel_residual = -1.0;
  if (st != ENKF_SUCCESS) return st;
  st = diag_factor();
  if (st != ENKF_SUCCESS) return st;
  if (!info) return ENKF_SUCCESS;
  st = diag_solve(nrhs, D, ldd, Z, ldz);
  return st != ENKF_SUCCESS ? st : get_info(info);
}

// ------------------------------------------------------------------ blocked
// Panel p covers levels k0 .. k0+bl-1. With U holding R^{-1} V updated by the
// panels before p:  P = V_K^T [U_K, U_rest];  M = I + P[:, :bl] = L D L^T;
// U_rest -= U_K (M^{-1} P[:, bl:]).
enkf_status Plan::factor_blocked() {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  const size_t wes = dtype_size(wdt);
  enkf_status st;
  if (mixed) {
    st = launch_convert(n, N, static_cast<const double*>(V), ldv, static_cast<float*>(Vw), ldu, nullptr, nullptr,
                        nullptr, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  const void* Vk = vwork();
  const int64_t ldvk = ldvw();
  {
    if (block_r) {
      st = block_step1(wdt, N, Vk, ldvk, U, ldu);
    } else {
      TimedLaunch tl(&timing, stream, KC_STEP1, 2.0 * n * N * wes + 8.0 * n, (double)n * N);
      st = launch_scale_rows(wdt, n, N, Vk, ldvk, r, U, ldu, status, stream);
    }
    if (st != ENKF_SUCCESS) return st;
  }
  for (int p = 0; p < npanel; ++p) {
    const int k0 = p * block;
    const int bl = std::min(block, N - k0);
    const int mrest = N - k0 - bl;
    const void* VK = static_cast<const char*>(Vk) + (size_t)k0 * ldvk * wes;
    const void* UK = static_cast<const char*>(U) + (size_t)k0 * ldu * wes;
    void* Ur = static_cast<char*>(U) + (size_t)(k0 + bl) * ldu * wes;
    {
      TimedLaunch tl(&timing, stream, KC_GRAM, (double)(2 * bl + mrest) * n * wes, 2.0 * n * bl * (bl + mrest));
      st = panel_tn(n, bl, bl + mrest, VK, ldvk, UK, ldu, Pbuf, bl);
      if (st != ENKF_SUCCESS) return st;
    }
    {
      TimedLaunch tl(&timing, stream, KC_PANEL_FACTOR, 0.0, (double)bl * bl * bl + 2.0 * bl * bl * mrest);
      st = launch_panel_factor(bl, Pbuf, bl, gamma + k0, Sfac + (size_t)p * block * block, status, stream);
      if (st != ENKF_SUCCESS) return st;
      st = launch_panel_apply(bl, mrest, Sfac + (size_t)p * block * block, Pbuf + (size_t)bl * bl, bl, Qbuf, stream);
      if (st != ENKF_SUCCESS) return st;
    }
    if (mrest > 0) {
      NnArgs a{};
      a.bws = Bt;
      a.n = n;
      a.K = bl;
      a.m = mrest;
      a.A = UK;
      a.lda = ldu;
      a.Bm = Qbuf;
      a.ldb = bl;
      a.scale = 1.0;
      a.Cin = Ur;
      a.ldc = ldu;
      a.Cout = Ur;
      a.ldo = ldu;
      TimedLaunch tl(&timing, stream, KC_PANEL_UPDATE, (double)(bl + 2 * mrest) * n * wes, 2.0 * n * bl * mrest);
      st = panel_nn(a);
      if (st != ENKF_SUCCESS) return st;
    }
  }
  return ENKF_SUCCESS;
}

// Z = W^{-1} D in the working type (D may be Z itself).
enkf_status Plan::solve_blocked(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool step1_done,
                                double* z64, int64_t ldz64, bool z64_acc, const double* z64_sumsq) {
  if (z64 && wdt != ENKF_F32) return fail(ENKF_ERR_NOT_SUPPORTED, "solve_blocked: FP64 destination needs FP32 panels");
  const int64_t n = desc.n_obs;
  const size_t wes = dtype_size(wdt);
  enkf_status st;
  if (nrhs == 0) return ENKF_SUCCESS;
  if (!step1_done) {
    TimedLaunch tl(&timing, stream, KC_STEP1, 2.0 * n * nrhs * wes + 8.0 * n, (double)n * nrhs);
    st = block_r ? launch_block_solve(wdt, max_bs, nblk, nrhs, boff, bpoff, Lf, D, ldd, Z, ldz, stream)
                 : launch_scale_rows(wdt, n, nrhs, D, ldd, r, Z, ldz, status, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  const void* Vk = vwork();
  const int64_t ldvk = ldvw();
  for (int p = 0; p < npanel; ++p) {
    const int k0 = p * block;
    const int bl = std::min(block, desc.n_ens - k0);
    const void* VK = static_cast<const char*>(Vk) + (size_t)k0 * ldvk * wes;
    const void* UK = static_cast<const char*>(U) + (size_t)k0 * ldu * wes;
    {
      TimedLaunch tl(&timing, stream, KC_GRAM, (double)(bl + nrhs) * n * wes, 2.0 * n * bl * nrhs);
      st = panel_tn(n, bl, nrhs, VK, ldvk, Z, ldz, Pbuf, bl);
      if (st != ENKF_SUCCESS) return st;
    }
    {
      TimedLaunch tl(&timing, stream, KC_PANEL_FACTOR, 0.0, 2.0 * bl * bl * nrhs);
      st = launch_panel_apply(bl, nrhs, Sfac + (size_t)p * block * block, Pbuf, bl, Qbuf, stream);
      if (st != ENKF_SUCCESS) return st;
    }
    NnArgs a{};
    a.bws = Bt;
    a.n = n;
    a.K = bl;
    a.m = nrhs;
    a.A = UK;
    a.lda = ldu;
    a.Bm = Qbuf;
    a.ldb = bl;
    a.scale = 1.0;
    a.Cin = Z;
    a.ldc = ldz;
    a.Cout = Z;
    a.ldo = ldz;
    if (z64 && p == npanel - 1) {                 // the last panel: the result goes to z64 in FP64
      a.Z64 = z64;
      a.ldz64 = ldz64;
      a.z64_acc = z64_acc ? 1 : 0;
      a.z64_sumsq = z64_sumsq;
      TimedLaunch tl(&timing, stream, KC_PANEL_UPDATE,
                     (double)(bl + nrhs) * n * wes + (z64_acc ? 16.0 : 8.0) * n * nrhs, 2.0 * n * bl * nrhs);
      st = desc.math == ENKF_MATH_F32 ? launch_nn(ENKF_F32, NN_UPDATE64, a, stream)
                                      : launch_nn_lowp(desc.math, NN_UPDATE64, a, stream);
      if (st != ENKF_SUCCESS) return st;
      continue;
    }
    TimedLaunch tl(&timing, stream, KC_PANEL_UPDATE, (double)(bl + 2 * nrhs) * n * wes, 2.0 * n * bl * nrhs);
    st = panel_nn(a);
    if (st != ENKF_SUCCESS) return st;
  }
  return ENKF_SUCCESS;
}

// Mixed precision: Z0 = W~^{-1} D with FP32 panels, then Z += W~^{-1} rho
// with rho = D - (R Z + V (V^T Z)) formed in FP64. The narrowing copy of D
// or rho also applies R^{-1} (Step 1), so the panels start from it. Inputs
// with the FP32 exponent range (FP32, BF16 parts) take R^{-1} rho straight
// from the residual product. The FP16 forms divide every right-hand side by
// the rms of R^{-1} times it (norms[2]) before narrowing and multiply the
// correction back, so neither a large R^{-1} D nor a shrinking residual
// leaves the FP16 range; they keep the FP64 copy of rho for that.
enkf_status Plan::solve_mixed(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool sync) {
  const int64_t n = desc.n_obs;
  last.refine_iters = 0;
  last.rel_residual = -1.0;
  if (nrhs == 0) return ENKF_SUCCESS;
  float* W = static_cast<float*>(Zw);
  const bool fp16 = desc.math == ENKF_MATH_F16 || desc.math == ENKF_MATH_F16X2;
  double* scale = fp16 ? norms + kNrmScale : nullptr;
  enkf_status st;
  if (fp16) {
    st = launch_sumsq(n, nrhs, static_cast<const double*>(D), ldd, r, norms + kNrmPart, scale, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  st = launch_convert(n, nrhs, static_cast<const double*>(D), ldd, W, ldu, scale, r, status, stream);
  if (st != ENKF_SUCCESS) return st;
  // the last panel update of each solve writes (or adds) its result to Z in
  // FP64 itself (the FP16 forms times the scale they divided by), so the
  // correction is never stored in FP32 for a separate widening pass
  double* Zd = static_cast<double*>(Z);
  st = solve_blocked(nrhs, W, ldu, W, ldu, true, Zd, ldz, false, scale);
  if (st != ENKF_SUCCESS) return st;
  const int maxit = desc.refine_max_iter;
  for (int it = 0; it <= maxit; ++it) {
    if (!sync && it == maxit) break;
    st = residual64(nrhs, D, ldd, Z, ldz, it == 0, fp16 ? nullptr : W);
    if (st != ENKF_SUCCESS) return st;
    if (sync) {
      double h[2];
      ENKF_HIP_CHECK(hipMemcpyAsync(h, norms, sizeof(h), hipMemcpyDeviceToHost, stream));
      ENKF_HIP_CHECK(hipStreamSynchronize(stream));
      last.rel_residual = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
      if (last.rel_residual <= desc.refine_tol || it == maxit) break;
    }
    if (fp16) {
      st = launch_sumsq(n, nrhs, rho, ldu, r, norms + kNrmPart, scale, stream);
      if (st != ENKF_SUCCESS) return st;
      st = launch_convert(n, nrhs, rho, ldu, W, ldu, scale, r, status, stream);
      if (st != ENKF_SUCCESS) return st;
    }
    st = solve_blocked(nrhs, W, ldu, W, ldu, true, Zd, ldz, true, scale);
    if (st != ENKF_SUCCESS) return st;
    last.refine_iters = it + 1;
  }
  return ENKF_SUCCESS;
}

// FP64 blocked solve refined with FP64 residuals and FP64 blocked
// corrections: Z = W~^{-1} D, then Z += W~^{-1} rho.
enkf_status Plan::solve_refined64(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool sync) {
  const int64_t n = desc.n_obs;
  last.refine_iters = 0;
  last.rel_residual = -1.0;
  if (nrhs == 0) return ENKF_SUCCESS;
  enkf_status st = solve_blocked(nrhs, D, ldd, Z, ldz);
  if (st != ENKF_SUCCESS) return st;
  const int maxit = desc.refine_max_iter;
  for (int it = 0; it <= maxit; ++it) {
    if (!sync && it == maxit) break;
    st = residual64(nrhs, D, ldd, Z, ldz, it == 0);
    if (st != ENKF_SUCCESS) return st;
    if (sync) {
      double h[2];
      ENKF_HIP_CHECK(hipMemcpyAsync(h, norms, sizeof(h), hipMemcpyDeviceToHost, stream));
      ENKF_HIP_CHECK(hipStreamSynchronize(stream));
      last.rel_residual = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
      if (last.rel_residual <= desc.refine_tol || it == maxit) break;
    }
    st = solve_blocked(nrhs, rho, ldu, rho, ldu);
    if (st != ENKF_SUCCESS) return st;
    st = launch_add(n, nrhs, rho, ldu, static_cast<double*>(Z), ldz, stream);
    if (st != ENKF_SUCCESS) return st;
    last.refine_iters = it + 1;
  }
  return ENKF_SUCCESS;
}

// rho = D - (r o Z + V (V^T Z)) in FP64 and the squared norms of rho and
// (d_norm) D.
enkf_status Plan::residual64(int nrhs, const void* D, int64_t ldd, const void* Z, int64_t ldz, bool d_norm,
                             float* w32) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  enkf_status st;
  {
    TimedLaunch tl(&timing, stream, KC_RESIDUAL_TN, (double)(N + nrhs) * n * 8.0, 2.0 * n * N * nrhs);
    st = launch_tn(ENKF_F64, n, N, nrhs, V, ldv, Z, ldz, G, N, tn_part, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  {
    NnArgs a{};
    a.bws = Bt;
    a.n = n;
    a.K = N;
    a.m = nrhs;
    a.A = V;
    a.lda = ldv;
    a.Bm = G;
    a.ldb = N;
    a.scale = 1.0;
    a.Cin = Z;
    a.ldc = ldz;
    a.Cout = rho;
    a.ldo = ldu;
    a.Cout32 = w32;
    a.ldo32 = ldu;
    a.Din = D;
    a.ldd = ldd;
    a.r = r;
    a.part = res_part;            // ||rho||^2 (the convergence test and the scale
    a.part_cap = res_part_cap;    // of rho) from the kernel's own outputs
    a.sumsq = norms;
    // bytes: V, Z and D read, rho written in FP64, or R^{-1} rho in FP32 (w32)
    TimedLaunch tl(&timing, stream, KC_RESIDUAL,
                   (double)(N + 2 * nrhs) * n * 8.0 + (double)nrhs * n * (w32 ? 4.0 : 8.0) + 8.0 * n,
                   2.0 * n * N * nrhs);
    st = launch_nn(ENKF_F64, NN_RESIDUAL, a, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  // ||D||^2, constant over the solve
  if (!d_norm) return ENKF_SUCCESS;
  return launch_sumsq(n, nrhs, static_cast<const double*>(D), ldd, nullptr, norms + kNrmPart, norms + kNrmD, stream);
}

// ------------------------------------------------------------------ common
// A fill kernel rather than a memset, so the sequence stays valid under
// stream capture.
enkf_status Plan::clear_status() {
  clear_words_kernel<<<1, 64, 0, stream>>>(status, 1);
  ENKF_HIP_CHECK(hipGetLastError());
  return ENKF_SUCCESS;
}

enkf_status Plan::read_status(unsigned* st) {
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  ENKF_HIP_CHECK(hipMemcpy(st, status, sizeof(unsigned), hipMemcpyDeviceToHost));
  return ENKF_SUCCESS;
}

enkf_status Plan::solve(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info) {
  enkf_status st;
  if (desc.algo == ENKF_SM_PLAIN) {
    st = solve_plain(nrhs, D, ldd, Z, ldz);
    last.refine_iters = 0;
    last.rel_residual = -1.0;
  } else if (mixed) {
    st = solve_mixed(nrhs, D, ldd, Z, ldz, info != nullptr);
  } else if (refine64) {
    st = solve_refined64(nrhs, D, ldd, Z, ldz, info != nullptr);
  } else {
    st = solve_blocked(nrhs, D, ldd, Z, ldz);
    last.refine_iters = 0;
    last.rel_residual = -1.0;
  }
  if (st != ENKF_SUCCESS) return st;
  if (info) {
    st = diag_solve(nrhs, D, ldd, Z, ldz);
    if (st != ENKF_SUCCESS) return st;
    st = get_info(info);
    if (st != ENKF_SUCCESS) return st;
    if ((mixed || refine64) && desc.refine_tol > 0.0 && nrhs > 0 && !(last.rel_residual <= desc.refine_tol))
    {
      char buf[96];
      snprintf(buf, sizeof(buf), "refinement stopped at relative residual %.3e after %d steps", last.rel_residual,
               last.refine_iters);
      return fail(ENKF_ERR_NO_CONVERGENCE, buf);
    }
  }
  return ENKF_SUCCESS;
}

enkf_status Plan::analysis(int64_t n_state, enkf_dtype x_dtype, enkf_math math, const void* XB, int64_t ldx,
                           const void* Z, int64_t ldz, void* XA, int64_t ldxa) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  {
    TimedLaunch tl(&timing, stream, KC_GRAM, 2.0 * (double)n * N * es, 2.0 * (double)n * N * N);
    enkf_status st = launch_tn(desc.dtype, n, N, N, V, ldv, Z, ldz, G, N, tn_part, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  NnArgs a{};
    a.bws = Bt;
  a.n = n_state;
  a.K = N;
  a.m = N;
  a.A = XB;
  a.lda = ldx;
  a.Bm = G;
  a.ldb = N;
  a.scale = 1.0 / std::sqrt((double)(N - 1));
  a.Cin = XB;
  a.ldc = ldx;
  a.Cout = XA;
  a.ldo = ldxa;
  const size_t xes = dtype_size(x_dtype);
  TimedLaunch tl(&timing, stream, KC_ANALYSIS, 2.0 * (double)n_state * N * xes, 2.0 * (double)n_state * N * N);
  if (math == ENKF_MATH_F64 || math == ENKF_MATH_F32) return launch_nn(x_dtype, NN_ANALYSIS, a, stream);
  return launch_nn_lowp(math, NN_ANALYSIS, a, stream);
}

enkf_status Plan::get_info(enkf_sm_info* info) {
  unsigned st = 0;
  enkf_status e = read_status(&st);
  if (e != ENKF_SUCCESS) return e;
  enkf_sm_info out = last;
  out.gamma_min = std::numeric_limits<double>::infinity();
  out.gamma_max = -std::numeric_limits<double>::infinity();
  double g[256];   // the pivots, a chunk at a time (no host allocation)
  for (int k0 = 0; k0 < desc.n_ens; k0 += 256) {
    const int cnt = std::min(256, desc.n_ens - k0);
    ENKF_HIP_CHECK(hipMemcpy(g, gamma + k0, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    for (int k = 0; k < cnt; ++k) {
      out.gamma_min = std::min(out.gamma_min, g[k]);
      out.gamma_max = std::max(out.gamma_max, g[k]);
    }
  }
  out.device_status = (int32_t)st;
  out.hip_error = (int32_t)hipPeekAtLastError();
  out.block = desc.algo == ENKF_SM_BLOCKED ? block : 1;
  *info = out;
  if (st != 0)
    return fail(static_cast<enkf_status>(st), "a kernel latched an error (r_i or gamma_k not finite or not > 0)");
  return ENKF_SUCCESS;
}

enkf_status Plan::get_pivots(double* gamma_host, int32_t* perm_host) {
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  ENKF_HIP_CHECK(hipMemcpy(gamma_host, gamma, sizeof(double) * desc.n_ens, hipMemcpyDeviceToHost));
  if (perm_host) {
    if (pivot) ENKF_HIP_CHECK(hipMemcpy(perm_host, perm, sizeof(int32_t) * desc.n_ens, hipMemcpyDeviceToHost));
    else
      for (int k = 0; k < desc.n_ens; ++k) perm_host[k] = k;
  }
  return ENKF_SUCCESS;
}

}  // namespace enkf
