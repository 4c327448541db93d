// On-box throughput of the matrix cores, the measured counterpart of the
// published peaks that the rooflines divide by. Every wave issues a long run
// of independent MFMAs on register operands (no memory traffic); the kernel's
// rate is what the part sustains for that input type at its running clock.
#include "enkf_internal.h"
#include "mfma_common.h"

namespace enkf {
namespace {

constexpr int CAL_NT = 256;   // 4 waves
constexpr int CAL_ACC = 8;    // independent accumulators per wave

template <typename MF>
__device__ __forceinline__ typename MF::op_t cal_operand(int l);

template <>
__device__ __forceinline__ double cal_operand<MfmaF64>(int l) { return 1e-3 * (1 + l % 7); }
template <>
__device__ __forceinline__ float cal_operand<MfmaF32>(int l) { return 1e-3f * (1 + l % 7); }
template <>
__device__ __forceinline__ mf_bf8 cal_operand<MfmaBF16>(int l) {
  mf_bf8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (__bf16)(1e-3f * (1 + (l + e) % 7));
  return v;
}
template <>
__device__ __forceinline__ mf_h8 cal_operand<MfmaF16>(int l) {
  mf_h8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (_Float16)(1e-3f * (1 + (l + e) % 7));
  return v;
}

// Two waves per SIMD at least: with the default budget (eight) the FP64
// accumulators do not fit the VGPRs, and the compiler copies them to and from
// the accumulation registers around every group of MFMAs.
template <typename MF>
__global__ __launch_bounds__(CAL_NT, 2) void mfma_loop_kernel(int iters, float* __restrict__ out) {
  const int l = threadIdx.x % kWave;
  const typename MF::op_t a = cal_operand<MF>(l), b = cal_operand<MF>(l + 3);
  typename MF::acc_t acc[CAL_ACC];
#pragma unroll
  for (int i = 0; i < CAL_ACC; ++i) acc[i] = MF::zero();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CAL_ACC; ++i) acc[i] = MF::mma(a, b, acc[i]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CAL_ACC; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += (float)acc[i][r];
  // the sum is used, so the loop is kept; it is never negative
  if (s < 0.f) out[0] = s;
}

template <typename MF>
enkf_status time_loop(double flops_per_mfma, double* tflops) {
  int dev = 0, cus = 0;
  ENKF_HIP_CHECK(hipGetDevice(&dev));
  ENKF_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = cus * 8;                     // 8 waves per SIMD
  const int iters = 4096;
  float* out = nullptr;
  ENKF_HIP_CHECK(hipMalloc(&out, sizeof(float)));
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  enkf_status st = ENKF_SUCCESS;
  float ms = 0.f;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = fail(ENKF_ERR_HIP, "mfma peak: stream or event creation failed");
  } else {
    mfma_loop_kernel<MF><<<blocks, CAL_NT, 0, s>>>(iters, out);   // warm-up (clocks, code load)
    (void)hipEventRecord(e0, s);
    mfma_loop_kernel<MF><<<blocks, CAL_NT, 0, s>>>(iters, out);
    (void)hipEventRecord(e1, s);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f))
      st = fail(ENKF_ERR_HIP, "mfma peak: timing failed");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  if (st != ENKF_SUCCESS) return st;
  const double mfmas = (double)blocks * (CAL_NT / kWave) * iters * CAL_ACC;
  *tflops = mfmas * flops_per_mfma / (ms * 1e-3) / 1e12;
  return ENKF_SUCCESS;
}

}  // namespace
}  // namespace enkf

extern "C" enkf_status enkf_mfma_peak(enkf_math math, double* tflops) {
  using namespace enkf;
  if (!tflops) return fail(ENKF_ERR_INVALID_ARG, "mfma_peak: NULL result");
  switch (math) {
    case ENKF_MATH_F64: return time_loop<MfmaF64>(2.0 * 16 * 16 * 4, tflops);
    case ENKF_MATH_F32: return time_loop<MfmaF32>(2.0 * 16 * 16 * 4, tflops);
    case ENKF_MATH_BF16: return time_loop<MfmaBF16>(2.0 * 16 * 16 * 32, tflops);
    case ENKF_MATH_F16: return time_loop<MfmaF16>(2.0 * 16 * 16 * 32, tflops);
    default: return fail(ENKF_ERR_NOT_SUPPORTED, "mfma_peak: math must be F64, F32, BF16 or F16");
  }
}
