// VALU issue rates of the MI355X, for the roofline of the evaluation
// kernels (a measurement probe run by bench.py --valu-rates; not part of
// the evaluation path and not linked into libwl.so).
//
// Each kernel keeps 8 independent dependency chains per lane of one
// instruction class, on 8 waves per SIMD over the whole chip, so that the
// SIMDs issue back to back:
//   fp32   v_fma_f32                     (8 per iteration)
//   trans  v_rsq_f32, v_exp_f32, v_rcp_f32, v_log_f32 in turn
//                                        (4 per chain, 32 per iteration)
//   fp64   v_fma_f64                     (8 per iteration)
// The chains' values stay finite or settle on fixed points (the rates do not
// depend on the operands), and every result feeds one store so that nothing
// is dead.  Rate = wave-instructions issued over the chip per second.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_rate_fp32(float* __restrict__ out, int iters,
                                                      float b, float c) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1e-3f * (float)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], b, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_rate_trans(float* __restrict__ out, int iters) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1.0f + 1e-3f * (float)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float r = __builtin_amdgcn_rsqf(a[j]);
      const float e = __builtin_amdgcn_exp2f(-r);
      const float q = __builtin_amdgcn_rcpf(e);
      a[j] = __builtin_amdgcn_logf(q);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_rate_fp64(double* __restrict__ out, int iters,
                                                      double b, double c) {
  double a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1e-3 * (double)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fma(a[j], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += a[j];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// Measures the three rates on the current device: rates[0..2] = FP32 FMA,
// transcendental and FP64 FMA wave-instructions per second over the chip
// (best of `reps` timed launches each, after one warm-up); ms[0..2] the
// best launch durations.  n_cu: compute units (8 waves per SIMD are
// launched on each).  Returns 0, or the HIP error code.
int wl_probe_valu_rates(int n_cu, int reps, double* rates, double* ms) {
  const int64_t n_blocks = (int64_t)n_cu * 4 * 8 * 64 / kBlock;
  const int64_t n_threads = n_blocks * kBlock;
  const double n_waves = (double)n_threads / 64.0;
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, n_threads * sizeof(double));
  if (e != hipSuccess) return (int)e;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  const int iters[3] = {1 << 18, 1 << 14, 1 << 16};
  const double per_iter[3] = {8.0, 32.0, 8.0};
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    float best = 1e30f;
    for (int r = -1; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(t0, nullptr);
      if (k == 0)
        hipLaunchKernelGGL(k_rate_fp32, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[0], 0.999f, 1e-3f);
      else if (k == 1)
        hipLaunchKernelGGL(k_rate_trans, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[1]);
      else
        hipLaunchKernelGGL(k_rate_fp64, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (double*)buf, iters[2], 0.999, 1e-3);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float m = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&m, t0, t1);
      if (r >= 0 && m < best) best = m;
    }
    ms[k] = best;
    rates[k] = n_waves * iters[k] * per_iter[k] / (best * 1e-3);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(buf);
  return (int)e;
}

}  // extern "C"
