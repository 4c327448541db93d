// Internal declarations shared by the HIP sources of the library (not part
// of the C ABI). gfx950 (CDNA4) only: wave64, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "enkf_sm.h"

namespace enkf {

constexpr int kWave = 64;

// Device status word values (a subset of enkf_status).
constexpr unsigned kStatusNotSpd = ENKF_ERR_NOT_SPD;

// Kernel classes whose launches can be timed with HIP events (measurement).
enum KernelClass : int {
  KC_INIT_SWEEP = 0,   // plain: U-updates, one launch per level
  KC_SOLVE_SWEEP = 1,  // plain: Z-updates, one launch per level
  KC_BUILD = 2,        // V, D from the ensemble
  KC_ANALYSIS = 3,     // X^A = X^B + S G (tall GEMM incl. mean)
  KC_GRAM = 4,         // split-K products V^T X (analysis G, residual, panels)
  KC_PANEL_UPDATE = 5, // blocked: X -= U_K Q (+ look-ahead products)
  KC_PANEL_FACTOR = 6, // blocked: b x b LDL^T and solves
  KC_RESIDUAL = 7,     // FP64 residual of the refinement: D - (r o Z + V G)
  KC_STEP1 = 8,        // Step 1 (R^{-1} V, R^{-1} D) and the plain form's first products
  KC_FUSED_SWEEP = 9,  // plain: U- and Z-updates of one level in one launch (factor + solve)
  KC_LOCALIZE = 10,    // partially localized analysis update
  KC_RESIDUAL_TN = 11, // FP64 residual of the refinement: the product G = V^T Z
  KC_COUNT = 12
};

void set_error(const std::string& msg);
enkf_status fail(enkf_status s, const std::string& msg);
const char* status_name(enkf_status s);

#define ENKF_HIP_CHECK(expr)                                                              \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return ::enkf::fail(ENKF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Raises a kernel's dynamic-LDS limit to `bytes` once per device (the
// attribute belongs to the kernel on the current device); `done` holds one
// bit per device index below 64 (larger indices set it on every call).
inline enkf_status set_dynamic_lds(std::atomic<uint64_t>& done, const void* kernel, size_t bytes,
                                   const char* what) {
  int dev = 0;
  ENKF_HIP_CHECK(hipGetDevice(&dev));
  const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return ENKF_SUCCESS;
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    return fail(ENKF_ERR_HIP, what);
  done.fetch_or(bit, std::memory_order_release);
  return ENKF_SUCCESS;
}

// Records event pairs around launches of one kernel class and accumulates the
// algorithmic bytes and flops those launches move (measurement only).
struct Timing {
  bool enabled = false;
  struct Rec { int cls; hipEvent_t a, b; double bytes, flops; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double ms[KC_COUNT] = {};
  double bytes[KC_COUNT] = {};
  double flops[KC_COUNT] = {};
  int64_t launches[KC_COUNT] = {};
  hipEvent_t get_event();
  void begin(hipStream_t s, int cls, double bytes, double flops, hipEvent_t* a);
  void end(hipStream_t s, hipEvent_t a, int cls, double bytes, double flops);
  hipError_t harvest();  // synchronises on the recorded events
  void reset();
  ~Timing();
};

// RAII-free scope helper used around launches.
struct TimedLaunch {
  Timing* t; hipStream_t s; int cls; double by, fl; hipEvent_t a = nullptr;
  TimedLaunch(Timing* t_, hipStream_t s_, int c, double b, double f) : t(t_), s(s_), cls(c), by(b), fl(f) {
    if (t && t->enabled) t->begin(s, cls, by, fl, &a);
  }
  ~TimedLaunch() { if (t && t->enabled && a) t->end(s, a, cls, by, fl); }
};

// ---------------------------------------------------------------- plain sweeps
// One level pass (or Step 1) over `m` columns of X. See level_kernels.hip.
// The look-ahead products of a launch are left as per-block partials
// ([column][row block] layout); every block of the next launch sums the
// partials it needs itself, in row-block order, so no cross-block
// synchronisation is needed inside a launch.
struct LevelArgs {
  int64_t n;
  int vw;                               // elements per lane load (1, or 16 bytes' worth)
  void* X; int64_t ldx; int m;          // active columns X[:, 0..m)
  const void* uk;                       // u_k^{(k-1)} (level) or nullptr (Step 1)
  const double* gamma_in;               // solve: &gamma[k]; factorisation: nullptr (formed from prev)
  double* gamma_out;                    // factorisation: &gamma[k] written by block (0,0)
  const double* prev;                   // partials of the previous launch ([col][nb]) or nullptr
  int prev_m;                           // columns in prev
  int prev_off;                         // active column q uses prev column q + prev_off
  const void* vnext;                    // v_{k+1} or nullptr (no look-ahead products)
  const double* r;                      // Step 1: diag(R)
  const void* src; int64_t lds;         // Step 1: V or D
  double* part_out;                     // this launch's partials ([m][nb])
  void* dst; int64_t ldo;               // if set, the updated columns go here instead of back to X
  // pivoting: active column q is column colmap[q] of X (and partial slot
  // colmap[q]); u_k = uk + (*uk_idx) ldu_idx and v_{k+1} = vnext + (*vn_idx)
  // ldv_idx, read on the device (the pivots are chosen on the device)
  const int32_t* colmap;
  const int32_t* uk_idx; int64_t ldu_idx;
  const int32_t* vn_idx; int64_t ldv_idx;
  unsigned* status;                     // device status word
};

enkf_status launch_level(enkf_dtype dt, const LevelArgs& a, hipStream_t s);

// The plain factorisation and/or solve of a small FP64 system in one block
// (the columns and V resident in the LDS); see small_sweep.hip.
// Scale of a residual block: its root mean square (1 when it is zero or
// when no sum of squares is given). The FP16 refinement divides the
// narrowed right-hand side by it and multiplies the correction back.
__device__ __forceinline__ double rms_scale(const double* sumsq, double count) {
  if (!sumsq) return 1.0;
  const double s = sqrt(sumsq[0] / count);
  return (s > 0.0 && s < 1e300) ? s : 1.0;
}

struct SmallSweepArgs {
  int64_t n;
  int N, nrhs;
  const double* r;
  const double* V; int64_t ldv;
  const double* D; int64_t ldd;
  double* U; int64_t ldu;                 // U columns at their levels (the plan's factor), written
  const double* Uin;                      // solve with a stored factor (ldu): u_k and gamma_k read, U not written
  double* Z; int64_t ldz;                 // may alias D (D is read before Z is written)
  double* gamma;                          // the N pivots
  unsigned* status;
};
constexpr size_t kSmallSweepMaxLds = 56 * 1024;   // dynamic LDS: with the 8 KiB of h_k, the default 64 KiB
constexpr int64_t kSmallSweepMaxRows = 1024;       // rows of h_k
size_t small_sweep_lds_bytes(int64_t n, int N, int nrhs);
enkf_status launch_small_sweep(const SmallSweepArgs& a, hipStream_t s);
// gamma[k] = 1 + sum of column `col` of partials (last level of a factorisation).
enkf_status launch_gamma_from_partials(const double* part, int nb, int col, double* gamma_out, unsigned* status,
                                       hipStream_t s);
int level_row_blocks(enkf_dtype dt, int vw, int64_t n);
int level_vw(enkf_dtype dt);

// ---------------------------------------------------------------- pivoting
struct PivotArgs {
  int init;                 // 1: from the diagonal partials; 0: before level k
  int k, N, nz;             // level, members, Z columns appended to the active list
  const double* part; int nb;   // partials [slot][nb]
  int32_t* perm;            // perm[k] = column used at level k
  double* gamma;            // gamma[k]
  double* gcur;             // candidate pivots (N)
  double* cbuf;             // c_i of this level (N)
  const int32_t* rem_in;    // remaining columns before level k (N - k)
  int32_t* rem_out;         // remaining after level k (N - k - 1), or 0..N-1 (init)
  int32_t* act_out;         // active list of level k (N - k - 1 + nz)
  unsigned* status;
};
enkf_status launch_diag_partials(enkf_dtype dt, int64_t n, int N, const void* V, int64_t ldv, const double* r,
                                 int nb, double* part, hipStream_t s);
enkf_status launch_pivot(const PivotArgs& a, hipStream_t s);

// ---------------------------------------------------------------- block-diagonal R
constexpr int kMaxRBlock = ENKF_MAX_R_BLOCK;
// R_b = L L^T for every block (off: row offsets, poff: packed offsets, both
// nblk + 1, device); Y = R^{-1} X block by block (FP64 arithmetic).
enkf_status launch_block_chol(int64_t nblk, const int64_t* off, const int64_t* poff, const double* Rb, double* Lf,
                              unsigned* status, hipStream_t s);
enkf_status launch_block_solve(enkf_dtype dt, int max_bs, int64_t nblk, int m, const int64_t* off,
                               const int64_t* poff, const double* Lf, const void* X, int64_t ldx, void* Y, int64_t ldy,
                               hipStream_t s);

// ---------------------------------------------------------------- partial localization
struct LocalizeArgs {
  int64_t n_state, n_obs;
  int N;
  const void* XB; int64_t ldx;
  const void* V; int64_t ldv;
  const void* Z; int64_t ldz;
  const int64_t* loc;        // state index of each observation (device)
  double length;             // e-folding distance (> 0)
  int64_t radius;            // impact is zero past this distance; < 0: no cut-off
  int64_t ring;              // distances on a ring of this many points; 0: no wrap
  void* XA; int64_t ldxa;
};
enkf_status launch_localize(enkf_dtype dt, const LocalizeArgs& a, hipStream_t s);

// ---------------------------------------------------------------- build
enkf_status launch_build_vd(enkf_dtype dt, int64_t n_state, int n_ens, const void* XB, int64_t ldx,
                            const int64_t* obs_idx, int64_t n_obs, const double* y, const void* E, int64_t lde,
                            void* V, void* D, int64_t ldv, hipStream_t s);

}  // namespace enkf
