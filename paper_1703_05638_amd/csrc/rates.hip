// Attainable float64 arithmetic rates of the device, measured with operands
// in registers only: v_mfma_f64_16x16x4f64 (the instruction of the float64
// Gram, projection and sine-transform kernels) and the vector FMA.  The
// published peaks assume the nominal clock; these give the rate the matrix
// and vector units reach under a sustained load of each, which is what the
// float64 kernels can approach at best.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace lrp {
namespace {

typedef double rate_d4 __attribute__((ext_vector_type(4)));
constexpr int kRateThreads = 256;
constexpr int kRateBlocks = 256 * 8;  // eight workgroups per compute unit
constexpr int kRateAcc = 8;           // independent accumulator tiles per wave
constexpr int kRateChains = 16;       // independent FMA chains per lane

__global__ __launch_bounds__(kRateThreads) void k_rate_mfma_f64(int iters, double* __restrict__ out) {
  rate_d4 acc[kRateAcc];
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
#pragma unroll
  for (int i = 0; i < kRateAcc; ++i) acc[i] = rate_d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kRateAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kRateAcc; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(long)blockIdx.x * kRateThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kRateThreads) void k_rate_fma_f64(int iters, double* __restrict__ out) {
  double x[kRateChains];
  const double b = 1.0 - 1e-12 * threadIdx.x, c = 1e-13;
#pragma unroll
  for (int i = 0; i < kRateChains; ++i) x[i] = 1.0 + 1e-3 * i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kRateChains; ++i) x[i] = __builtin_fma(x[i], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kRateChains; ++i) s += x[i];
  out[(long)blockIdx.x * kRateThreads + threadIdx.x] = s;
}

}  // namespace

void measure_fp64_rates(int iters, double* mfma_tflops, double* valu_tflops) {
  if (iters < 1 || iters > 100000) fail(LRPOST_EINVAL, "rate probe: iterations must be in 1..100000");
  double* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
  };
  try {
    LRP_HIP(hipMalloc(&out, sizeof(double) * kRateBlocks * kRateThreads));
    LRP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    LRP_HIP(hipEventCreate(&e0));
    LRP_HIP(hipEventCreate(&e1));
    // best of three timed launches after one untimed one
    auto best_ms = [&](auto kernel) {
      float best = 0.f;
      for (int rep = 0; rep < 4; ++rep) {
        LRP_HIP(hipEventRecord(e0, st));
        hipLaunchKernelGGL(kernel, dim3(kRateBlocks), dim3(kRateThreads), 0, st, iters, out);
        LRP_HIP(hipGetLastError());
        LRP_HIP(hipEventRecord(e1, st));
        LRP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        LRP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep == 1 || (rep > 1 && ms < best)) best = ms;
      }
      return (double)best;
    };
    const double waves = kRateBlocks * (kRateThreads / 64.0);
    // one 16 x 16 x 4 product is 2048 flops per wave
    const double mfma_flops = 2048.0 * kRateAcc * iters * waves;
    const double fma_flops = 2.0 * kRateChains * iters * (double)kRateBlocks * kRateThreads;
    *mfma_tflops = mfma_flops / best_ms(k_rate_mfma_f64) / 1e9;
    *valu_tflops = fma_flops / best_ms(k_rate_fma_f64) / 1e9;
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

}  // namespace lrp
