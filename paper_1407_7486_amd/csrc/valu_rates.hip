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
//   mix    1 transcendental + 4 v_fma_f32 per chain (40 per iteration)
//   vop2   v_fmac_f32, v_mul_f32 or v_add_f32 with VGPR operands (8 per
//          iteration)
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

// Two-operand (VOP2) forms with a VGPR operand: v_fmac_f32 (MODE 0),
// v_mul_f32 (1), v_add_f32 (2), 8 per iteration.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_rate_vop2(float* __restrict__ out, int iters,
                                                      float b, float c) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1e-3f * (float)(threadIdx.x + j);
  // lane-varying operands, so that they live in VGPRs
  const float bv = b + 1e-9f * (float)threadIdx.x;
  const float cv = c + 1e-9f * (float)threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (MODE == 0) a[j] = fmaf(bv, cv, a[j]);
      else if (MODE == 1) a[j] = a[j] * bv;
      else a[j] = a[j] + cv;
    }
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

// Mixed stream: per chain and iteration one transcendental (rsq, exp, rcp
// and log in turn over four iterations' worth of chains) and 4 FP32 FMAs,
// the ratio of the evaluation kernel's sech^2 segment (4 transcendentals,
// ~15 other operations).  If the transcendental unit overlapped the FP32
// pipe, an iteration would take less than the sum of its parts' times.
__global__ __launch_bounds__(kBlock) void k_rate_mix(float* __restrict__ out, int iters,
                                                     float b, float c) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1.0f + 1e-3f * (float)(threadIdx.x + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float t;
      if (j % 4 == 0) t = __builtin_amdgcn_rsqf(a[j]);
      else if (j % 4 == 1) t = __builtin_amdgcn_exp2f(-a[j]);
      else if (j % 4 == 2) t = __builtin_amdgcn_rcpf(a[j]);
      else t = __builtin_amdgcn_logf(a[j]);
      t = fmaf(t, b, c);
      t = fmaf(t, b, c);
      t = fmaf(t, b, c);
      a[j] = fmaf(t, b, 1.0f);
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

// Measures the rates on the current device: rates[0..6] = FP32 FMA (VOP3,
// SGPR operand), transcendental, FP64 FMA, mixed stream (1 transcendental :
// 4 FMA), v_fmac_f32, v_mul_f32 and v_add_f32 (VOP2) wave-instructions per
// second over the chip (best of `reps` timed launches each, after one
// warm-up); ms[0..6] the best launch durations.  n_cu: compute units (8
// waves per SIMD are launched on each).  Returns 0, or the HIP error code.
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
  const int iters[7] = {1 << 18, 1 << 14, 1 << 16, 1 << 15, 1 << 18, 1 << 18, 1 << 18};
  const double per_iter[7] = {8.0, 32.0, 8.0, 40.0, 8.0, 8.0, 8.0};
  for (int k = 0; k < 7 && e == hipSuccess; ++k) {
    float best = 1e30f;
    for (int r = -1; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(t0, nullptr);
      if (k == 0)
        hipLaunchKernelGGL(k_rate_fp32, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[0], 0.999f, 1e-3f);
      else if (k == 1)
        hipLaunchKernelGGL(k_rate_trans, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[1]);
      else if (k == 2)
        hipLaunchKernelGGL(k_rate_fp64, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (double*)buf, iters[2], 0.999, 1e-3);
      else if (k == 3)
        hipLaunchKernelGGL(k_rate_mix, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[3], 0.999f, 1e-3f);
      else if (k == 4)
        hipLaunchKernelGGL(k_rate_vop2<0>, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[4], 0.999f, 1e-3f);
      else if (k == 5)
        hipLaunchKernelGGL(k_rate_vop2<1>, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[5], 0.999f, 1e-3f);
      else
        hipLaunchKernelGGL(k_rate_vop2<2>, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters[6], 0.999f, 1e-3f);
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
