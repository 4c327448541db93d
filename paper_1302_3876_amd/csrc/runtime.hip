// C ABI entry points: argument validation on the host, plan and workspace,
// launch sequencing on the caller's stream, device status word, timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "enkf_internal.h"
#include "plan.h"

namespace enkf {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

enkf_status fail(enkf_status s, const std::string& msg) {
  g_last_error = std::string(status_name(s)) + ": " + msg;
  return s;
}

const char* status_name(enkf_status s) {
  switch (s) {
    case ENKF_SUCCESS: return "success";
    case ENKF_ERR_INVALID_ARG: return "invalid argument";
    case ENKF_ERR_NOT_SPD: return "not positive definite";
    case ENKF_ERR_NO_CONVERGENCE: return "refinement did not converge";
    case ENKF_ERR_HIP: return "HIP runtime error";
    case ENKF_ERR_OUT_OF_MEMORY: return "out of memory";
    case ENKF_ERR_NOT_SUPPORTED: return "not supported";
  }
  return "unknown status";
}

// ------------------------------------------------------------------ timing
hipEvent_t Timing::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Timing::begin(hipStream_t s, int, double, double, hipEvent_t* a) {
  *a = get_event();
  if (*a) (void)hipEventRecord(*a, s);
}

void Timing::end(hipStream_t s, hipEvent_t a, int cls, double by, double fl) {
  hipEvent_t b = get_event();
  if (!b) return;
  (void)hipEventRecord(b, s);
  pending.push_back({cls, a, b, by, fl});
}

hipError_t Timing::harvest() {
  for (auto& r : pending) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return e;
    float ms_ = 0.f;
    e = hipEventElapsedTime(&ms_, r.a, r.b);
    if (e != hipSuccess) return e;
    ms[r.cls] += ms_;
    bytes[r.cls] += r.bytes;
    flops[r.cls] += r.flops;
    launches[r.cls] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  return hipSuccess;
}

void Timing::reset() {
  for (int i = 0; i < KC_COUNT; ++i) { ms[i] = bytes[i] = flops[i] = 0.0; launches[i] = 0; }
}

Timing::~Timing() {
  for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : pool) (void)hipEventDestroy(e);
}

size_t dtype_size(enkf_dtype d) { return d == ENKF_F64 ? 8 : 4; }

static bool math_matches_plain(const enkf_sm_desc& d) {
  return (d.dtype == ENKF_F64 && d.math == ENKF_MATH_F64) || (d.dtype == ENKF_F32 && d.math == ENKF_MATH_F32);
}

enkf_status validate_desc(const enkf_sm_desc* d) {
  if (!d) return fail(ENKF_ERR_INVALID_ARG, "desc is NULL");
  if (d->n_obs < 1) return fail(ENKF_ERR_INVALID_ARG, "n_obs must be >= 1");
  if (d->n_ens < 1) return fail(ENKF_ERR_INVALID_ARG, "n_ens must be >= 1");
  if (d->dtype != ENKF_F64 && d->dtype != ENKF_F32) return fail(ENKF_ERR_INVALID_ARG, "unknown dtype");
  if (d->algo != ENKF_SM_PLAIN && d->algo != ENKF_SM_BLOCKED) return fail(ENKF_ERR_INVALID_ARG, "unknown algo");
  if (d->math < ENKF_MATH_F64 || d->math > ENKF_MATH_F16X2) return fail(ENKF_ERR_INVALID_ARG, "unknown math");
  if (d->flags & ~(ENKF_FLAG_PIVOT | ENKF_FLAG_DIAGNOSE | ENKF_FLAG_AUTOTUNE))
    return fail(ENKF_ERR_INVALID_ARG, "unknown flag bits");
  if (d->max_nrhs < 0) return fail(ENKF_ERR_INVALID_ARG, "max_nrhs must be >= 0");
  if (d->refine_max_iter < 0) return fail(ENKF_ERR_INVALID_ARG, "refine_max_iter must be >= 0");
  if (!(d->refine_tol >= 0.0)) return fail(ENKF_ERR_INVALID_ARG, "refine_tol must be >= 0");
  if (d->algo == ENKF_SM_PLAIN) {
    if (!math_matches_plain(*d))
      return fail(ENKF_ERR_INVALID_ARG, "plain algorithm: math must equal the storage type (F64/F64 or F32/F32)");
    if (d->block != 0 && d->block != 1) return fail(ENKF_ERR_INVALID_ARG, "plain algorithm: block must be 0 or 1");
  } else {
    if (d->block < 0 || d->block > d->n_ens) return fail(ENKF_ERR_INVALID_ARG, "block must be in [0, n_ens]");
    if (d->flags & ENKF_FLAG_PIVOT) return fail(ENKF_ERR_NOT_SUPPORTED, "pivoting is available for the plain algorithm");
    if (d->dtype == ENKF_F32 && d->math == ENKF_MATH_F64)
      return fail(ENKF_ERR_INVALID_ARG, "math F64 needs F64 storage");
  }
  return ENKF_SUCCESS;
}

// D and Z of a solve: the plain and the unrefined blocked solves run in
// place (Z == D with the same leading dimension); the refined and mixed
// solves read D again for every residual, so they need it untouched and take
// no overlap at all. Any other overlap of the two column ranges is refused.
enkf_status check_rhs_overlap(const Plan* p, const char* where, int32_t nrhs, const void* D, int64_t ldd,
                              const void* Z, int64_t ldz) {
  const size_t es = dtype_size(p->desc.dtype);
  const uintptr_t d0 = (uintptr_t)D, d1 = d0 + ((size_t)ldd * (nrhs - 1) + p->desc.n_obs) * es;
  const uintptr_t z0 = (uintptr_t)Z, z1 = z0 + ((size_t)ldz * (nrhs - 1) + p->desc.n_obs) * es;
  if (!(z0 < d1 && d0 < z1)) return ENKF_SUCCESS;
  if (p->mixed || p->refine64)
    return fail(ENKF_ERR_INVALID_ARG, std::string(where) + ": Z overlaps D, and a refined solve reads D after writing Z");
  if (D != Z || ldd != ldz)
    return fail(ENKF_ERR_INVALID_ARG, std::string(where) + ": Z overlaps D other than in place with the same leading dimension");
  return ENKF_SUCCESS;
}

}  // namespace enkf

using namespace enkf;

// ------------------------------------------------------------------ ABI
extern "C" {

enkf_status enkf_sm_validate_desc(const enkf_sm_desc* desc) { return validate_desc(desc); }

const char* enkf_status_string(enkf_status s) { return status_name(s); }

const char* enkf_last_error_message(void) { return g_last_error.c_str(); }

enkf_status enkf_build_vd(int64_t n_state, int32_t n_ens, enkf_dtype dtype, const void* XB, int64_t ldx,
                          const int64_t* obs_idx, int64_t n_obs, const double* y, const void* E, int64_t lde, void* V,
                          void* D, int64_t ldv, void* stream) {
  if (n_state < 1 || n_obs < 1) return fail(ENKF_ERR_INVALID_ARG, "build_vd: n_state and n_obs must be >= 1");
  if (n_ens < 2) return fail(ENKF_ERR_INVALID_ARG, "build_vd: n_ens must be >= 2 (S divides by sqrt(N-1))");
  if (dtype != ENKF_F64 && dtype != ENKF_F32) return fail(ENKF_ERR_INVALID_ARG, "build_vd: unknown dtype");
  if (ldx < n_state || lde < n_obs || ldv < n_obs) return fail(ENKF_ERR_INVALID_ARG, "build_vd: leading dimension too small");
  if (!XB || !obs_idx || !y || !E || !V || !D) return fail(ENKF_ERR_INVALID_ARG, "build_vd: NULL pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return launch_build_vd(dtype, n_state, n_ens, XB, ldx, obs_idx, n_obs, y, E, lde, V, D, ldv, s);
}

enkf_status enkf_sm_init(enkf_sm_plan* out, const enkf_sm_desc* desc, const double* r, const void* V, int64_t ldv,
                         void* stream) {
  if (!out) return fail(ENKF_ERR_INVALID_ARG, "init: out is NULL");
  *out = nullptr;
  enkf_status st = validate_desc(desc);
  if (st != ENKF_SUCCESS) return st;
  if (!r || !V) return fail(ENKF_ERR_INVALID_ARG, "init: r or V is NULL");
  if (ldv < desc->n_obs) return fail(ENKF_ERR_INVALID_ARG, "init: ldv < n_obs");
  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(ENKF_ERR_OUT_OF_MEMORY, "init: plan");
  st = p->create(*desc, r, V, ldv, static_cast<hipStream_t>(stream));
  if (st != ENKF_SUCCESS) {
    delete p;
    return st;
  }
  st = p->tune_block();
  if (st == ENKF_SUCCESS) st = p->factor();
  if (st != ENKF_SUCCESS) {
    delete p;
    return st;
  }
  *out = reinterpret_cast<enkf_sm_plan>(p);
  return ENKF_SUCCESS;
}

enkf_status enkf_sm_init_block_r(enkf_sm_plan* out, const enkf_sm_desc* desc, const enkf_block_r* R, const void* V,
                                 int64_t ldv, void* stream) {
  if (!out) return fail(ENKF_ERR_INVALID_ARG, "init_block_r: out is NULL");
  *out = nullptr;
  enkf_status st = validate_desc(desc);
  if (st != ENKF_SUCCESS) return st;
  if (!R || !R->offsets || !R->blocks || !V) return fail(ENKF_ERR_INVALID_ARG, "init_block_r: NULL argument");
  if (ldv < desc->n_obs) return fail(ENKF_ERR_INVALID_ARG, "init_block_r: ldv < n_obs");
  if (R->n_blocks < 1 || R->offsets[0] != 0 || R->offsets[R->n_blocks] != desc->n_obs)
    return fail(ENKF_ERR_INVALID_ARG, "init_block_r: offsets must run from 0 to n_obs");
  for (int64_t b = 0; b < R->n_blocks; ++b) {
    const int64_t sz = R->offsets[b + 1] - R->offsets[b];
    if (sz < 1) return fail(ENKF_ERR_INVALID_ARG, "init_block_r: offsets must increase");
    if (sz > ENKF_MAX_R_BLOCK) return fail(ENKF_ERR_NOT_SUPPORTED, "init_block_r: block larger than ENKF_MAX_R_BLOCK");
  }
  if (desc->flags & ENKF_FLAG_PIVOT) return fail(ENKF_ERR_NOT_SUPPORTED, "init_block_r: pivoting needs a diagonal R");
  if (desc->algo == ENKF_SM_BLOCKED &&
      (desc->math != (desc->dtype == ENKF_F64 ? ENKF_MATH_F64 : ENKF_MATH_F32) || desc->refine_max_iter > 0))
    return fail(ENKF_ERR_NOT_SUPPORTED, "init_block_r: the refinement residual needs a diagonal R");
  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(ENKF_ERR_OUT_OF_MEMORY, "init: plan");
  st = p->create(*desc, nullptr, V, ldv, static_cast<hipStream_t>(stream));
  if (st == ENKF_SUCCESS) st = p->set_block_r(R->n_blocks, R->offsets);
  if (st == ENKF_SUCCESS) st = p->factor_block_r(R->blocks);
  if (st == ENKF_SUCCESS) st = p->tune_block();
  if (st == ENKF_SUCCESS) st = p->factor();
  if (st != ENKF_SUCCESS) {
    delete p;
    return st;
  }
  *out = reinterpret_cast<enkf_sm_plan>(p);
  return ENKF_SUCCESS;
}

enkf_status enkf_sm_refactor_block_r(enkf_sm_plan plan, const double* R_blocks, const void* V, int64_t ldv) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "refactor_block_r: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p->block_r) return fail(ENKF_ERR_INVALID_ARG, "refactor_block_r: the plan has a diagonal R");
  if (!R_blocks || !V) return fail(ENKF_ERR_INVALID_ARG, "refactor_block_r: NULL argument");
  if (ldv < p->desc.n_obs) return fail(ENKF_ERR_INVALID_ARG, "refactor_block_r: ldv < n_obs");
  p->V = V;
  p->ldv = ldv;
  enkf_status st = p->clear_status();
  if (st == ENKF_SUCCESS) st = p->factor_block_r(R_blocks);
  return st == ENKF_SUCCESS ? p->factor() : st;
}

enkf_status enkf_sm_refactor(enkf_sm_plan plan, const double* r, const void* V, int64_t ldv) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "refactor: plan is NULL");
  if (!r || !V) return fail(ENKF_ERR_INVALID_ARG, "refactor: r or V is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (p->block_r) return fail(ENKF_ERR_INVALID_ARG, "refactor: the plan has a block-diagonal R (enkf_sm_refactor_block_r)");
  if (ldv < p->desc.n_obs) return fail(ENKF_ERR_INVALID_ARG, "refactor: ldv < n_obs");
  p->r = r;
  p->V = V;
  p->ldv = ldv;
  enkf_status st = p->clear_status();
  if (st != ENKF_SUCCESS) return st;
  return p->factor();
}

enkf_status enkf_sm_solve(enkf_sm_plan plan, int32_t nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz,
                          enkf_sm_info* info) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "solve: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (nrhs < 0 || nrhs > p->max_nrhs) return fail(ENKF_ERR_INVALID_ARG, "solve: nrhs outside [0, max_nrhs]");
  if (nrhs > 0) {
    if (!D || !Z) return fail(ENKF_ERR_INVALID_ARG, "solve: D or Z is NULL");
    if (ldd < p->desc.n_obs || ldz < p->desc.n_obs) return fail(ENKF_ERR_INVALID_ARG, "solve: leading dimension < n_obs");
    enkf_status st = check_rhs_overlap(p, "solve", nrhs, D, ldd, Z, ldz);
    if (st != ENKF_SUCCESS) return st;
  }
  return p->solve(nrhs, D, ldd, Z, ldz, info);
}

enkf_status enkf_sm_factor_solve(enkf_sm_plan plan, const double* r, const void* V, int64_t ldv, int32_t nrhs,
                                 const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: plan is NULL");
  if (!r || !V) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: r or V is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (p->block_r) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: the plan has a block-diagonal R");
  if (ldv < p->desc.n_obs) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: ldv < n_obs");
  if (nrhs < 0 || nrhs > p->max_nrhs) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: nrhs outside [0, max_nrhs]");
  if (nrhs > 0) {
    if (!D || !Z) return fail(ENKF_ERR_INVALID_ARG, "factor_solve: D or Z is NULL");
    if (ldd < p->desc.n_obs || ldz < p->desc.n_obs)
      return fail(ENKF_ERR_INVALID_ARG, "factor_solve: leading dimension < n_obs");
    enkf_status st = check_rhs_overlap(p, "factor_solve", nrhs, D, ldd, Z, ldz);
    if (st != ENKF_SUCCESS) return st;
  }
  p->r = r;
  p->V = V;
  p->ldv = ldv;
  enkf_status st = p->clear_status();
  if (st != ENKF_SUCCESS) return st;
  return p->factor_solve(nrhs, D, ldd, Z, ldz, info);
}

static enkf_status analysis_checks(Plan* p, int64_t n_state, enkf_dtype x_dtype, const void* XB, int64_t ldx,
                                   const void* Z, int64_t ldz, void* XA, int64_t ldxa) {
  if (n_state < 1) return fail(ENKF_ERR_INVALID_ARG, "analysis: n_state must be >= 1");
  if (p->desc.n_ens < 2) return fail(ENKF_ERR_INVALID_ARG, "analysis: n_ens must be >= 2");
  if (!XB || !Z || !XA) return fail(ENKF_ERR_INVALID_ARG, "analysis: NULL pointer");
  if (ldx < n_state || ldxa < n_state || ldz < p->desc.n_obs)
    return fail(ENKF_ERR_INVALID_ARG, "analysis: leading dimension too small");
  const size_t es = dtype_size(x_dtype);
  const uintptr_t xb0 = (uintptr_t)XB, xb1 = xb0 + ((size_t)ldx * (p->desc.n_ens - 1) + n_state) * es;
  const uintptr_t xa0 = (uintptr_t)XA, xa1 = xa0 + ((size_t)ldxa * (p->desc.n_ens - 1) + n_state) * es;
  if (xa0 < xb1 && xb0 < xa1) return fail(ENKF_ERR_INVALID_ARG, "analysis: XA overlaps XB");
  return ENKF_SUCCESS;
}

enkf_status enkf_analysis(enkf_sm_plan plan, int64_t n_state, const void* XB, int64_t ldx, const void* Z, int64_t ldz,
                          void* XA, int64_t ldxa) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "analysis: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  enkf_status st = analysis_checks(p, n_state, p->desc.dtype, XB, ldx, Z, ldz, XA, ldxa);
  if (st != ENKF_SUCCESS) return st;
  const enkf_math math = p->desc.dtype == ENKF_F64 ? ENKF_MATH_F64 : ENKF_MATH_F32;
  return p->analysis(n_state, p->desc.dtype, math, XB, ldx, Z, ldz, XA, ldxa);
}

enkf_status enkf_localized_analysis(enkf_sm_plan plan, int64_t n_state, const void* XB, int64_t ldx, const void* Z,
                                    int64_t ldz, const int64_t* obs_loc, double length, int64_t radius, int64_t ring,
                                    void* XA, int64_t ldxa) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "localized analysis: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  enkf_status st = analysis_checks(p, n_state, p->desc.dtype, XB, ldx, Z, ldz, XA, ldxa);
  if (st != ENKF_SUCCESS) return st;
  if (!obs_loc) return fail(ENKF_ERR_INVALID_ARG, "localized analysis: obs_loc is NULL");
  if (!(length > 0.0) || !std::isfinite(length))
    return fail(ENKF_ERR_INVALID_ARG, "localized analysis: length must be finite and > 0");
  if (ring != 0 && ring < n_state) return fail(ENKF_ERR_INVALID_ARG, "localized analysis: ring must be 0 or >= n_state");
  LocalizeArgs a{};
  a.n_state = n_state;
  a.n_obs = p->desc.n_obs;
  a.N = p->desc.n_ens;
  a.XB = XB;
  a.ldx = ldx;
  a.V = p->V;
  a.ldv = p->ldv;
  a.Z = Z;
  a.ldz = ldz;
  a.loc = obs_loc;
  a.length = length;
  a.radius = radius;
  a.ring = ring;
  a.XA = XA;
  a.ldxa = ldxa;
  const double N = p->desc.n_ens, ns = (double)n_state, no = (double)p->desc.n_obs;
  const double chunks = std::ceil(N / 128.0);
  TimedLaunch tl(&p->timing, p->stream, KC_LOCALIZE, 2.0 * ns * N * p->es + 2.0 * no * N * p->es,
                 4.0 * ns * no * N);
  (void)chunks;
  return launch_localize(p->desc.dtype, a, p->stream);
}

enkf_status enkf_analysis_ex(enkf_sm_plan plan, int64_t n_state, enkf_dtype x_dtype, enkf_math math, const void* XB,
                             int64_t ldx, const void* Z, int64_t ldz, void* XA, int64_t ldxa) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "analysis: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (x_dtype != ENKF_F64 && x_dtype != ENKF_F32) return fail(ENKF_ERR_INVALID_ARG, "analysis: unknown x_dtype");
  if (math < ENKF_MATH_F64 || math > ENKF_MATH_F16X2) return fail(ENKF_ERR_INVALID_ARG, "analysis: unknown math");
  if ((x_dtype == ENKF_F64) != (math == ENKF_MATH_F64))
    return fail(ENKF_ERR_INVALID_ARG, "analysis: FP64 ensembles take FP64 products; FP32 ensembles the others");
  enkf_status st = analysis_checks(p, n_state, x_dtype, XB, ldx, Z, ldz, XA, ldxa);
  if (st != ENKF_SUCCESS) return st;
  return p->analysis(n_state, x_dtype, math, XB, ldx, Z, ldz, XA, ldxa);
}

enkf_status enkf_sm_get_info(enkf_sm_plan plan, enkf_sm_info* info) {
  if (!plan || !info) return fail(ENKF_ERR_INVALID_ARG, "get_info: NULL argument");
  return reinterpret_cast<Plan*>(plan)->get_info(info);
}

enkf_status enkf_sm_get_tuning(enkf_sm_plan plan, int32_t* widths, double* ms, int32_t* count) {
  if (!plan || !count) return fail(ENKF_ERR_INVALID_ARG, "get_tuning: NULL argument");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  *count = p->ntune;
  for (int i = 0; i < p->ntune; ++i) {
    if (widths) widths[i] = p->tune_b[i];
    if (ms) ms[i] = p->tune_ms[i];
  }
  return ENKF_SUCCESS;
}

enkf_status enkf_sm_get_pivots(enkf_sm_plan plan, double* gamma_host, int32_t* perm_host) {
  if (!plan || !gamma_host) return fail(ENKF_ERR_INVALID_ARG, "get_pivots: NULL argument");
  return reinterpret_cast<Plan*>(plan)->get_pivots(gamma_host, perm_host);
}

void enkf_sm_destroy(enkf_sm_plan plan) {
  if (!plan) return;
  delete reinterpret_cast<Plan*>(plan);
}

enkf_status enkf_sm_set_timing(enkf_sm_plan plan, int32_t enable) {
  if (!plan) return fail(ENKF_ERR_INVALID_ARG, "set_timing: plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (p->timing.harvest() != hipSuccess) return fail(ENKF_ERR_HIP, "set_timing: event harvest failed");
  p->timing.reset();
  p->timing.enabled = enable != 0;
  return ENKF_SUCCESS;
}

enkf_status enkf_sm_get_timing(enkf_sm_plan plan, int32_t kernel_class, double* total_ms, int64_t* launches,
                               double* alg_bytes, double* alg_flops) {
  if (!plan || kernel_class < 0 || kernel_class >= KC_COUNT) return fail(ENKF_ERR_INVALID_ARG, "get_timing: bad argument");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (p->timing.harvest() != hipSuccess) return fail(ENKF_ERR_HIP, "get_timing: event harvest failed");
  if (total_ms) *total_ms = p->timing.ms[kernel_class];
  if (launches) *launches = p->timing.launches[kernel_class];
  if (alg_bytes) *alg_bytes = p->timing.bytes[kernel_class];
  if (alg_flops) *alg_flops = p->timing.flops[kernel_class];
  return ENKF_SUCCESS;
}

}  // extern "C"
