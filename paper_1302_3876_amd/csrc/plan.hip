// Plan: workspace layout and the launch sequences of the factorisation,
// solve and analysis.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "plan.h"

namespace enkf {

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

const void* Plan::vcol(int k) const {
  return static_cast<const char*>(V) + (size_t)k * (size_t)ldv * es;
}

enkf_status Plan::create(const enkf_sm_desc& d, const double* r_, const void* V_, int64_t ldv_, hipStream_t s) {
  desc = d;
  r = r_;
  V = V_;
  ldv = ldv_;
  stream = s;
  es = dtype_size(d.dtype);
  max_nrhs = d.max_nrhs > 0 ? d.max_nrhs : d.n_ens;
  if (d.algo != ENKF_SM_PLAIN) return fail(ENKF_ERR_NOT_SUPPORTED, "init: only the plain algorithm is available");
  if (d.flags & ENKF_FLAG_PIVOT) return fail(ENKF_ERR_NOT_SUPPORTED, "init: pivoting is not available yet");

  const int64_t n = d.n_obs;
  const int N = d.n_ens;
  const int mcols = std::max(N, max_nrhs);
  ldu = (int64_t)align_up((size_t)n, 64);

  // carve the workspace
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t oU = take((size_t)ldu * N * es);
  const size_t oGamma = take(sizeof(double) * N);
  const size_t part_elems = (size_t)level_row_blocks(d.dtype, 1, n) * mcols;
  const size_t oP0 = take(sizeof(double) * part_elems);
  const size_t oP1 = take(sizeof(double) * part_elems);
  const size_t oStat = take(sizeof(unsigned) * 4);
  const size_t oG = take(sizeof(double) * (size_t)N * N);
  const size_t oGP = take(sizeof(double) * (size_t)gram_partial_elems(n, N, N));
  ws_bytes = off;
  hipError_t e = hipMalloc(&ws, ws_bytes);
  if (e != hipSuccess) {
    ws = nullptr;
    return fail(ENKF_ERR_OUT_OF_MEMORY, "init: workspace of " + std::to_string(ws_bytes) + " bytes");
  }
  U = ws + oU;
  gamma = reinterpret_cast<double*>(ws + oGamma);
  part[0] = reinterpret_cast<double*>(ws + oP0);
  part[1] = reinterpret_cast<double*>(ws + oP1);
  status = reinterpret_cast<unsigned*>(ws + oStat);
  G = reinterpret_cast<double*>(ws + oG);
  gram_partial = reinterpret_cast<double*>(ws + oGP);
  // The status word starts at zero.
  ENKF_HIP_CHECK(hipMemsetAsync(ws + oStat, 0, sizeof(unsigned) * 4, stream));
  last.rel_residual = -1.0;
  return ENKF_SUCCESS;
}

Plan::~Plan() {
  if (stream || ws) (void)hipStreamSynchronize(stream);
  if (ws) (void)hipFree(ws);
}

enkf_status Plan::factor() { return factor_plain(); }

// Byte and flop model of one sweep launch over m columns of n rows:
// read and write the m columns, read u_k and v_{k+1} (Step 1: the source
// columns and r instead of u_k); flops 4 m n (update + look-ahead product).
static void sweep_model(int64_t n, int m, size_t es, bool step1, bool look, double* by, double* fl) {
  double cols = 2.0 * m + (look ? 1.0 : 0.0) + (step1 ? 0.0 : 1.0);
  *by = cols * (double)n * (double)es + (step1 ? 8.0 * (double)n : 0.0);
  *fl = (double)n * m * (look ? 4.0 : 2.0);
}

static bool vec_ok(const void* p, int64_t ld, int vw, size_t es) {
  return p == nullptr || (((uintptr_t)p % (vw * es)) == 0 && (ld % vw) == 0);
}

enkf_status Plan::factor_plain() {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  const int vw = (vec_ok(U, ldu, level_vw(desc.dtype), es) && vec_ok(V, ldv, level_vw(desc.dtype), es))
                     ? level_vw(desc.dtype) : 1;
  const int nb = level_row_blocks(desc.dtype, vw, n);
  // Step 1 for V: U0 = R^{-1} V and the products v_1^T u_j^{(0)}.
  LevelArgs a{};
  a.n = n;
  a.vw = vw;
  a.status = status;
  a.X = U;
  a.ldx = ldu;
  a.m = N;
  a.src = V;
  a.lds = ldv;
  a.r = r;
  a.vnext = vcol(0);
  a.part_out = part[0];
  {
    double by, fl;
    sweep_model(n, N, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_INIT_SWEEP, by, fl);
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
  const int w = level_vw(desc.dtype);
  const int vw = (vec_ok(U, ldu, w, es) && vec_ok(V, ldv, w, es) && vec_ok(D, ldd, w, es) && vec_ok(Z, ldz, w, es))
                     ? w : 1;
  LevelArgs a{};
  a.n = n;
  a.vw = vw;
  a.status = status;
  a.X = Z;
  a.ldx = ldz;
  a.m = nrhs;
  a.src = D;
  a.lds = ldd;
  a.r = r;
  a.vnext = vcol(0);
  a.part_out = part[0];
  {
    double by, fl;
    sweep_model(n, nrhs, es, true, true, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_SOLVE_SWEEP, by, fl);
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
    b.part_out = part[(k + 1) & 1];
    double by, fl;
    sweep_model(n, nrhs, es, false, b.vnext != nullptr, &by, &fl);
    TimedLaunch tl(&timing, stream, KC_SOLVE_SWEEP, by, fl);
    enkf_status st = launch_level(desc.dtype, b, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  return ENKF_SUCCESS;
}

namespace {
__global__ void clear_words_kernel(unsigned* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}
}  // namespace

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
  enkf_status st = solve_plain(nrhs, D, ldd, Z, ldz);
  if (st != ENKF_SUCCESS) return st;
  last.refine_iters = 0;
  last.rel_residual = -1.0;
  if (info) return get_info(info);
  return ENKF_SUCCESS;
}

enkf_status Plan::analysis(int64_t n_state, const void* XB, int64_t ldx, const void* Z, int64_t ldz, void* XA,
                           int64_t ldxa) {
  const int64_t n = desc.n_obs;
  const int N = desc.n_ens;
  {
    const double by = 2.0 * (double)n * N * es;
    const double fl = 2.0 * (double)n * N * N;
    TimedLaunch tl(&timing, stream, KC_GRAM, by, fl);
    enkf_status st = launch_gram(desc.dtype, n, N, N, V, ldv, Z, ldz, G, N, gram_partial, stream);
    if (st != ENKF_SUCCESS) return st;
  }
  const double by = 2.0 * (double)n_state * N * es;
  const double fl = 2.0 * (double)n_state * N * N;
  TimedLaunch tl(&timing, stream, KC_ANALYSIS, by, fl);
  return launch_analysis(desc.dtype, n_state, N, XB, ldx, G, 1.0 / std::sqrt((double)(N - 1)), XA, ldxa, stream);
}

enkf_status Plan::get_info(enkf_sm_info* info) {
  unsigned st = 0;
  enkf_status e = read_status(&st);
  if (e != ENKF_SUCCESS) return e;
  std::vector<double> g(desc.n_ens);
  ENKF_HIP_CHECK(hipMemcpy(g.data(), gamma, sizeof(double) * desc.n_ens, hipMemcpyDeviceToHost));
  enkf_sm_info out = last;
  out.gamma_min = *std::min_element(g.begin(), g.end());
  out.gamma_max = *std::max_element(g.begin(), g.end());
  out.device_status = (int32_t)st;
  *info = out;
  if (st != 0) return fail(static_cast<enkf_status>(st), "a kernel latched an error (r_i or gamma_k not finite or not > 0)");
  return ENKF_SUCCESS;
}

enkf_status Plan::get_pivots(double* gamma_host, int32_t* perm_host) {
  ENKF_HIP_CHECK(hipStreamSynchronize(stream));
  ENKF_HIP_CHECK(hipMemcpy(gamma_host, gamma, sizeof(double) * desc.n_ens, hipMemcpyDeviceToHost));
  if (perm_host)
    for (int k = 0; k < desc.n_ens; ++k) perm_host[k] = perm_h.empty() ? k : perm_h[k];
  return ENKF_SUCCESS;
}

}  // namespace enkf
