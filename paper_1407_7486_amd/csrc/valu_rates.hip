// VALU issue rates of the MI355X, for the roofline of the evaluation
// kernels (a measurement probe run by bench.py --valu-rates; not part of
// the evaluation path and not linked into libwl.so).
//
// Each kernel keeps 8 independent dependency chains per lane of one
// instruction form, on 8 waves per SIMD over the whole chip, so that the
// SIMDs issue back to back.  The forms (the instruction each chain step
// compiles to, checked in the gfx950 assembly of this file):
//    0  v_fma_f32 (VOP3), one SGPR operand
//    1  transcendentals v_rsq, v_exp, v_rcp, v_log in turn (4 per chain)
//    2  v_fma_f64
//    3  mixed stream: 1 transcendental + 4 v_fma_f32 per chain
//    4  v_fmac_f32 (VOP2), VGPR operands only
//    5  v_mul_f32 (VOP2), VGPR operands
//    6  v_add_f32 (VOP2), inline constant
//    7  v_fma_f32 (VOP3), VGPR operands only
//    8  v_fma_f32 (VOP3) with a negated operand
//    9  v_fmaak_f32 (VOP2 with a 32-bit literal)
//   10  v_mul_f32 (VOP2) with a literal
//   11  v_fmac_f32 (VOP2) with an SGPR operand
//   12  v_exp_f32 (VOP1)
//   13  v_exp_f32 (VOP3, negated operand)
// The chains' values stay finite or settle (the rates do not depend on the
// operands), and every result feeds one store so that nothing is dead.
// Rate = wave-instructions issued over the chip per second.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;
constexpr int kForms = 14;

template <int FORM>
__global__ __launch_bounds__(kBlock) void k_rate(float* __restrict__ out, int iters, float b,
                                                 float c) {
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = 1.0f + 1e-3f * (float)(threadIdx.x + j);
  // lane-varying operands, so that they live in VGPRs
  const float bv = b + 1e-9f * (float)threadIdx.x;
  const float cv = c + 1e-9f * (float)threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if constexpr (FORM == 0) {
        a[j] = fmaf(a[j], b, cv);
      } else if constexpr (FORM == 1) {
        const float r = __builtin_amdgcn_rsqf(a[j]);
        const float e = __builtin_amdgcn_exp2f(-r);
        const float q = __builtin_amdgcn_rcpf(e);
        a[j] = __builtin_amdgcn_logf(q);
      } else if constexpr (FORM == 3) {
        // per chain one transcendental (rsq, exp, rcp, log over the chains)
        // and 4 FMAs: the ratio of the sech^2 segment
        float t;
        if (j % 4 == 0) t = __builtin_amdgcn_rsqf(a[j]);
        else if (j % 4 == 1) t = __builtin_amdgcn_exp2f(-a[j]);
        else if (j % 4 == 2) t = __builtin_amdgcn_rcpf(a[j]);
        else t = __builtin_amdgcn_logf(a[j]);
        t = fmaf(t, b, c);
        t = fmaf(t, b, c);
        t = fmaf(t, b, c);
        a[j] = fmaf(t, b, 1.0f);
      } else if constexpr (FORM == 4) {
        a[j] = fmaf(bv, cv, a[j]);
      } else if constexpr (FORM == 5) {
        a[j] = a[j] * bv;
      } else if constexpr (FORM == 6) {
        a[j] = a[j] + 1.0f;
      } else if constexpr (FORM == 7) {
        a[j] = fmaf(a[j], bv, cv);
      } else if constexpr (FORM == 8) {
        a[j] = fmaf(-a[j], bv, cv);
      } else if constexpr (FORM == 9) {
        a[j] = fmaf(a[j], bv, 0.37f);
      } else if constexpr (FORM == 10) {
        a[j] = a[j] * 1.00001f;
      } else if constexpr (FORM == 11) {
        a[j] = fmaf(b, cv, a[j]);
      } else if constexpr (FORM == 12) {
        a[j] = __builtin_amdgcn_exp2f(a[j]);
      } else if constexpr (FORM == 13) {
        a[j] = __builtin_amdgcn_exp2f(-a[j]);
      }
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

typedef void (*RateFn)(float*, int, float, float);
const RateFn kFns[kForms] = {k_rate<0>, k_rate<1>, nullptr,    k_rate<3>,  k_rate<4>,
                             k_rate<5>, k_rate<6>, k_rate<7>,  k_rate<8>,  k_rate<9>,
                             k_rate<10>, k_rate<11>, k_rate<12>, k_rate<13>};

}  // namespace

extern "C" {

// Measures the rates of the forms above on the current device: rates[f] =
// wave-instructions per second over the chip (best of `reps` timed
// launches, after one warm-up), ms[f] the best launch duration; n_forms
// entries are filled (at most 14).  n_cu: compute units (8 waves per SIMD
// are launched on each).  Returns 0, or the HIP error code.
int wl_probe_valu_rates(int n_cu, int reps, int n_forms, double* rates, double* ms) {
  if (n_forms > kForms) n_forms = kForms;
  const int64_t n_blocks = (int64_t)n_cu * 4 * 8 * 64 / kBlock;
  const int64_t n_threads = n_blocks * kBlock;
  const double n_waves = (double)n_threads / 64.0;
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, n_threads * sizeof(double));
  if (e != hipSuccess) return (int)e;
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  for (int k = 0; k < n_forms && e == hipSuccess; ++k) {
    // instructions per chain step and iterations (transcendental forms
    // issue ~4x slower)
    const double per_iter = k == 1 ? 32.0 : k == 3 ? 40.0 : 8.0;
    const int iters = k == 1 ? (1 << 14) : (k == 3 || k == 12 || k == 13) ? (1 << 15)
                                                                          : (1 << 17);
    float best = 1e30f;
    for (int r = -1; r < reps && e == hipSuccess; ++r) {
      e = hipEventRecord(t0, nullptr);
      if (k == 2)
        hipLaunchKernelGGL(k_rate_fp64, dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (double*)buf, iters, 0.999, 1e-3);
      else
        hipLaunchKernelGGL(kFns[k], dim3((uint32_t)n_blocks), dim3(kBlock), 0, nullptr,
                           (float*)buf, iters, 0.999f, 1e-3f);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float m = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&m, t0, t1);
      if (r >= 0 && m < best) best = m;
    }
    ms[k] = best;
    rates[k] = n_waves * iters * per_iter / (best * 1e-3);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(buf);
  return (int)e;
}

}  // extern "C"
