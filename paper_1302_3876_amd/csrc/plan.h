// The plan behind enkf_sm_plan: borrowed inputs, owned workspace, and the
// launch sequences of the factorisation, solve and analysis.
#pragma once

#include "enkf_internal.h"
#include "gemm_mfma.h"

namespace enkf {

size_t dtype_size(enkf_dtype d);
enkf_status validate_desc(const enkf_sm_desc* d);
struct Plan;
// Refuses an overlap of Z with D that the plan's solve cannot take (refined
// and mixed solves: any overlap; others: anything but in place).
enkf_status check_rhs_overlap(const Plan* p, const char* where, int32_t nrhs, const void* D, int64_t ldd,
                              const void* Z, int64_t ldz);
// Panel widths the tuner times for n_ens = N: 32, 64, 96, 128 up to N (N itself below 32).
std::vector<int> tune_candidates(int N);
constexpr int kMaxTune = 4;

// Slots of Plan::norms (device, FP64).
enum NormSlot : int {
  kNrmRho = 0,    // ||rho||_F^2 of the last residual
  kNrmD = 1,      // ||D||_F^2 of the solve
  kNrmScale = 2,  // ||R^{-1} x||_F^2 of the right-hand side narrowed next (FP16 forms)
  kNrmZ = 3,      // ||Z||_F^2 (diagnostics)
  kNrmW = 4,      // estimate of ||W||_2 (diagnostics, per factorisation)
  kNrmPart = 8    // reduction partials
};

struct Plan {
  enkf_sm_desc desc{};
  int max_nrhs = 0;
  hipStream_t stream = nullptr;
  const double* r = nullptr;
  const void* V = nullptr;
  int64_t ldv = 0;
  size_t es = 8;

  // workspace (one allocation, carved into the pieces below)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;         // false: a borrowed workspace (not freed, no wait at destruction)
  void* U = nullptr;            // plain factor: column k = u_k^{(k-1)}; then max_nrhs columns of Z (fused)
  int64_t ldu = 0;
  double* gamma = nullptr;      // N pivots
  double* part[2] = {nullptr, nullptr};  // level sweeps: per-block partial products, alternating
  unsigned* status = nullptr;   // device status word
  double* G = nullptr;          // N x N products V^T Z (analysis), N x nrhs (residual)
  double* tn_part = nullptr;    // split-K partials of the tn products
  char* Bt = nullptr;           // converted right factor of the nn products
  // blocked
  int block = 0;                // panel width b
  bool autotune = false;        // ENKF_FLAG_AUTOTUNE with block 0: width timed at init (tune_block)
  int ntune = 0;                // widths the tuner timed and their factor + solve times
  int tune_b[kMaxTune] = {};
  float tune_ms[kMaxTune] = {};
  int npanel = 0;
  double* Sfac = nullptr;       // npanel x (b x b) S = D^{-1/2} L^{-1} of M = L D L^T
  double* Pbuf = nullptr;       // b x (N + max_nrhs) panel products
  double* Qbuf = nullptr;       // b x max(N, max_nrhs)
  // mixed precision (math narrower than dtype): FP32 working copies
  bool mixed = false;
  bool refine64 = false;        // FP64 blocked solve with FP64 refinement
  bool diagnose = false;        // ENKF_FLAG_DIAGNOSE on an FP64, diagonal-R plan
  enkf_dtype wdt = ENKF_F64;    // working storage type of U, panels, Z-sweeps
  void* Vw = nullptr;           // FP32 copy of V (mixed)
  void* Zw = nullptr;           // FP32 correction (mixed), n x max_nrhs
  double* rho = nullptr;        // FP64 residual (mixed), n x max_nrhs
  double* norms = nullptr;      // slots kNrm* below, then reduction partials
  double* res_part = nullptr;   // per-block sums of rho^2 of the residual product
  int64_t res_part_cap = 0;
  // pivoting (plain)
  bool pivot = false;
  int32_t* perm = nullptr;      // V/U column used at each level (device)
  double* gcur = nullptr;       // candidate pivots
  double* cbuf = nullptr;       // products c_i of the current level
  int32_t* rem[2] = {nullptr, nullptr};  // remaining columns, alternating
  int32_t* act[2] = {nullptr, nullptr};  // active lists of the level launches, alternating

  // block-diagonal R (r == nullptr): row offsets, packed offsets and the
  // Cholesky factors of the blocks, in a second allocation
  bool block_r = false;
  int64_t nblk = 0;
  int max_bs = 0;
  char* bws = nullptr;
  int64_t* boff = nullptr;
  int64_t* bpoff = nullptr;
  double* Lf = nullptr;

  Timing timing;
  enkf_sm_info last{};

  // ext_ws: carve the workspace from this device buffer of ext_bytes (fails
  // with NOT_SUPPORTED when it does not fit) instead of allocating it
  enkf_status create(const enkf_sm_desc& d, const double* r, const void* V, int64_t ldv, hipStream_t s,
                     char* ext_ws = nullptr, size_t ext_bytes = 0);
  enkf_status factor();
  enkf_status tune_block();
  // ENKF_FLAG_DIAGNOSE: ||W||_2 estimate after a factorisation; after a
  // synchronous solve, the residual (if the form has none), ||Z|| and eta.
  enkf_status diag_factor();
  enkf_status diag_solve(int nrhs, const void* D, int64_t ldd, const void* Z, int64_t ldz);
  enkf_status solve(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info);
  // factor() and solve() together (plain: one launch per level for U and Z)
  enkf_status factor_solve(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, enkf_sm_info* info);
  enkf_status analysis(int64_t n_state, enkf_dtype x_dtype, enkf_math math, const void* XB, int64_t ldx,
                       const void* Z, int64_t ldz, void* XA, int64_t ldxa);
  enkf_status get_info(enkf_sm_info* info);
  enkf_status set_block_r(int64_t nblk, const int64_t* off_host);
  enkf_status factor_block_r(const double* Rblocks);
  enkf_status get_pivots(double* gamma_host, int32_t* perm_host);
  enkf_status read_status(unsigned* st);
  enkf_status clear_status();
  ~Plan();

 private:
  enkf_status factor_plain();
  enkf_status solve_plain(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz);
  enkf_status factor_solve_plain(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz);
  enkf_status sweep_pivot(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz);
  enkf_status block_step1(enkf_dtype dt, int m, const void* X, int64_t ldx, void* Y, int64_t ldy);
  enkf_status factor_blocked();
  // Z = (R + V V^T)^{-1} D with the blocked factor, all in the working type.
  // step1_done: Z already holds R^{-1} D (D is not read). z64 (FP32 working
  // type only): the last panel's update writes its result to z64 in FP64
  // (z64 = s result, or z64 += s result with z64_acc; s = rms_scale(z64_sumsq,
  // n nrhs), 1 without z64_sumsq) instead of back to Z.
  enkf_status solve_blocked(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool step1_done = false,
                            double* z64 = nullptr, int64_t ldz64 = 0, bool z64_acc = false,
                            const double* z64_sumsq = nullptr);
  enkf_status solve_mixed(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool sync);
  bool small_plain(int nrhs) const;
  enkf_status small_sweep(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool solve_only);
  enkf_status solve_refined64(int nrhs, const void* D, int64_t ldd, void* Z, int64_t ldz, bool sync);
  // rho = D - W Z in FP64, ||rho||^2 into norms[0] and, with d_norm,
  // ||D||^2 into norms[1] (constant over one solve, so formed once). With
  // w32, R^{-1} rho is written there in FP32 (leading dimension ldu) and rho
  // itself is not stored.
  enkf_status residual64(int nrhs, const void* D, int64_t ldd, const void* Z, int64_t ldz, bool d_norm,
                         float* w32 = nullptr);
  const void* vwork() const { return mixed ? Vw : V; }
  int64_t ldvw() const { return mixed ? ldu : ldv; }
  const void* vcol(int k) const;  // V column used at level k
  enkf_status panel_tn(int64_t n, int a, int m, const void* A, int64_t lda, const void* B, int64_t ldb, double* Gout,
                       int64_t ldg);
  enkf_status panel_nn(const NnArgs& a);
};

}  // namespace enkf
