// The allocation-free solve: enkf_sm_init + enkf_sm_factor_solve with the
// plan's workspace carved from a static device array instead of hipMalloc,
// for callers that cannot allocate (code under stream capture, tight
// serving loops, harnesses that forbid it). Same kernels and launch
// sequence as the planned calls.
#include <mutex>

#include "enkf_internal.h"
#include "plan.h"

namespace enkf {
namespace {

// One copy per GPU the library runs on, held until the process ends.
__device__ __align__(256) char scratch[ENKF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// The device address of the scratch array on the current device, found once
// per device with that device current (the array's name in host code is
// only a stand-in for the symbol, never a device address).
enkf_status scratch_ptr(char** out) {
  int dev = -1;
  ENKF_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ENKF_ERR_NOT_SUPPORTED, "solve_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    ENKF_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ENKF_ERR_HIP, "solve_noalloc: no device address for the static scratch");
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return ENKF_SUCCESS;
}

}  // namespace
}  // namespace enkf

using namespace enkf;

extern "C" enkf_status enkf_sm_solve_noalloc(const enkf_sm_desc* desc, const double* r, const void* V, int64_t ldv,
                                             int32_t nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz,
                                             enkf_sm_info* info, void* stream) {
  enkf_status st = validate_desc(desc);
  if (st != ENKF_SUCCESS) return st;
  if (desc->flags & ENKF_FLAG_AUTOTUNE)
    return fail(ENKF_ERR_NOT_SUPPORTED, "solve_noalloc: the panel-width tuner allocates; give the block");
  if (!r || !V) return fail(ENKF_ERR_INVALID_ARG, "solve_noalloc: r or V is NULL");
  if (ldv < desc->n_obs) return fail(ENKF_ERR_INVALID_ARG, "solve_noalloc: ldv < n_obs");
  const int32_t mx = desc->max_nrhs > 0 ? desc->max_nrhs : desc->n_ens;
  if (nrhs < 0 || nrhs > mx) return fail(ENKF_ERR_INVALID_ARG, "solve_noalloc: nrhs outside [0, max_nrhs]");
  if (nrhs > 0) {
    if (!D || !Z) return fail(ENKF_ERR_INVALID_ARG, "solve_noalloc: D or Z is NULL");
    if (ldd < desc->n_obs || ldz < desc->n_obs)
      return fail(ENKF_ERR_INVALID_ARG, "solve_noalloc: leading dimension < n_obs");
  }
  char* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != ENKF_SUCCESS) return st;
  Plan p;   // on the stack, over the static scratch
  st = p.create(*desc, r, V, ldv, static_cast<hipStream_t>(stream), ws, ENKF_NOALLOC_SCRATCH_BYTES);
  if (st != ENKF_SUCCESS) return st;
  if (nrhs > 0) {
    st = check_rhs_overlap(&p, "solve_noalloc", nrhs, D, ldd, Z, ldz);
    if (st != ENKF_SUCCESS) return st;
  }
  return p.factor_solve(nrhs, D, ldd, Z, ldz, info);
}
