// Effective action from the group sums of an evaluation (Eq. cylEA for the
// rho_cm integral, Sec. 3.3 for the counterterms and the small-T series,
// Sec. 6 for Simpson's rule on x = 1/(1 + T/T_max), Sec. 4.2.3 for doing
// the integrals group by group).  FP64 throughout; sizes are small (G x
// n_rho x n_T), so one thread per (group, rho) integrates over T.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wl_host.h"

namespace wl {
namespace {

// eB(rho^2) of the field kinds (include/wl.h).
__device__ double field_b(int kind, double eB0, double lam, double r2) {
  switch (kind) {
    case WL_SECH2: {
      const double E = exp(-2.0 * sqrt(r2) / lam);
      const double d = 1.0 + E;
      return eB0 * 4.0 * E / (d * d);
    }
    case WL_GAUSS: return eB0 * exp(-r2 / (lam * lam));
    case WL_RATIONAL: {
      const double l2 = lam * lam, d = l2 + r2;
      return eB0 * l2 * l2 / (d * d);
    }
    default: return eB0;
  }
}

// Node t of the T grid (ascending, t = 0 is T = a) and its Simpson weight
// times the Jacobian T_max / x^2 of x = 1/(1 + T/T_max).
__device__ __forceinline__ void t_node(const wl_action_spec& sp, int32_t t, double& T,
                                       double& wj) {
  const double xa = 1.0 / (1.0 + sp.a / sp.T_max);
  const int32_t k = sp.n_T - t;  // x_k = k xa / n_T, k = n_T .. 1
  const double x = k * xa / sp.n_T;
  T = t == 0 ? sp.a : sp.T_max * (1.0 / x - 1.0);
  const double c = (k == sp.n_T) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
  wj = c * (xa / sp.n_T) / 3.0 * (sp.T_max / (x * x));
}

__device__ __forceinline__ void rho_node(const wl_action_spec& sp, int32_t j, double& rho,
                                         double& wj) {
  const int32_t k = sp.n_rho - j;  // x_k = k / n_rho
  const double x = (double)k / sp.n_rho;
  rho = j == 0 ? 0.0 : sp.rho_max * (1.0 / x - 1.0);
  const double c = (k == sp.n_rho) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
  wj = c * (1.0 / sp.n_rho) / 3.0 * (sp.rho_max / (x * x));
}

// Row r < G: group r's density from W = G S / N_l; row G: the LCF density
// (W = theta coth theta, or theta / sinh theta for scalars, theta = eB T).
__global__ __launch_bounds__(256) void k_action_density(
    wl_action_spec sp, int32_t kind, double eB0, double lam, int32_t spin,
    const double* __restrict__ sums, int32_t n_groups, int64_t n_loops,
    double* __restrict__ dens) {
  const int32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (n_groups + 1) * sp.n_rho) return;
  const int32_t r = id / sp.n_rho, j = id % sp.n_rho;
  double rho, wr;
  rho_node(sp, j, rho, wr);
  const double b = field_b(kind, eB0, lam, rho * rho);
  const double m2 = sp.m2, b4 = b * b * b * b, b6 = b4 * b * b;
  double c1, c2, c3, c4;  // small-T series (Eqs. fermI, scalI)
  if (spin) {
    c1 = -b4 / 45.0;
    c2 = b4 * m2 / 45.0;
    c3 = 2.0 * b6 / 945.0 - b4 * m2 * m2 / 90.0;
    c4 = (7.0 * b4 * m2 * m2 * m2 - 4.0 * b6 * m2) / 1890.0;
  } else {
    c1 = 7.0 * b4 / 360.0;
    c2 = -7.0 * b4 * m2 / 360.0;
    c3 = (147.0 * b4 * m2 * m2 - 31.0 * b6) / 15120.0;
    c4 = (31.0 * b6 * m2 - 49.0 * b4 * m2 * m2 * m2) / 15120.0;
  }
  const double a = sp.a, a2 = a * a;
  double acc = c1 * a2 / 2.0 + c2 * a2 * a / 3.0 + c3 * a2 * a2 / 4.0 + c4 * a2 * a2 * a / 5.0;
  const double scale = (double)n_groups / (double)n_loops;
  const double* srow = sums + ((int64_t)r * sp.n_rho + j) * sp.n_T;
  for (int32_t t = 0; t < sp.n_T; ++t) {
    double T, wt;
    t_node(sp, t, T, wt);
    const double th = b * T;
    double W;
    if (r < n_groups) {
      W = srow[t] * scale;
    } else if (th == 0.0) {
      W = 1.0;
    } else if (spin) {
      W = th / tanh(th);
    } else {
      W = th > 700.0 ? 0.0 : th / sinh(th);
    }
    const double counter = spin ? 1.0 + th * th / 3.0 : 1.0 - th * th / 6.0;
    acc += wt * (exp(-m2 * T) / (T * T * T)) * (W - counter);
  }
  dens[id] = acc;
}

// (1/4pi) int rho D drho per row; NaN for the constant field (divergent).
__global__ __launch_bounds__(256) void k_action_rho(wl_action_spec sp, int32_t kind,
                                                    int32_t n_rows,
                                                    const double* __restrict__ dens,
                                                    double* __restrict__ act) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  if (kind == WL_CONST) {
    act[r] = NAN;
    return;
  }
  double acc = 0.0;
  for (int32_t j = 0; j < sp.n_rho; ++j) {
    double rho, wr;
    rho_node(sp, j, rho, wr);
    acc += wr * rho * dens[(int64_t)r * sp.n_rho + j];
  }
  act[r] = acc / (4.0 * M_PI);
}

// Mean and standard error over the G group rows: thread j < n_rho for the
// densities, thread n_rho for the action.
__global__ __launch_bounds__(256) void k_action_stats(int32_t n_rho, int32_t n_groups,
                                                      const double* __restrict__ dens,
                                                      const double* __restrict__ act,
                                                      double* __restrict__ dmean,
                                                      double* __restrict__ derr,
                                                      double* __restrict__ amean_err) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > n_rho) return;
  const double* v = j < n_rho ? dens + j : act;
  const int64_t stride = j < n_rho ? n_rho : 1;
  double s = 0.0;
  for (int32_t g = 0; g < n_groups; ++g) s += v[g * stride];
  const double m = s / n_groups;
  double ss = 0.0;
  for (int32_t g = 0; g < n_groups; ++g) {
    const double d = v[g * stride] - m;
    ss += d * d;
  }
  const double e = n_groups > 1 ? sqrt(ss / ((double)n_groups * (n_groups - 1))) : NAN;
  if (j < n_rho) {
    dmean[j] = m;
    derr[j] = e;
  } else {
    amean_err[0] = m;
    amean_err[1] = e;
  }
}

}  // namespace

hipError_t launch_action(const wl_action_spec& sp, int32_t kind, double eB0, double lam,
                         int32_t spin, const double* d_sums, int32_t n_groups,
                         int64_t n_loops, double* d_dens, double* d_act, double* d_dmean,
                         double* d_derr, double* d_amean_err, hipStream_t stream) {
  const int32_t rows = n_groups + 1;
  const int32_t n1 = rows * sp.n_rho;
  hipLaunchKernelGGL(k_action_density, dim3((n1 + 255) / 256), dim3(256), 0, stream, sp,
                     kind, eB0, lam, spin, d_sums, n_groups, n_loops, d_dens);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_action_rho, dim3((rows + 255) / 256), dim3(256), 0, stream, sp, kind,
                     rows, d_dens, d_act);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_action_stats, dim3((sp.n_rho + 1 + 255) / 256), dim3(256), 0, stream,
                     sp.n_rho, n_groups, d_dens, d_act, d_dmean, d_derr, d_amean_err);
  return hipGetLastError();
}

}  // namespace wl

using namespace wl;

extern "C" {

int wl_action_grids(const wl_action_spec* sp, double* T, double* rho) {
  if (!sp || !T || !rho) return WL_EINVAL;
  if (!(sp->a > 0.0 && sp->T_max > 0.0 && sp->rho_max > 0.0 && isfinite(sp->a) &&
        isfinite(sp->T_max) && isfinite(sp->rho_max)) ||
      sp->n_T < 2 || sp->n_T % 2 || sp->n_rho < 2 || sp->n_rho % 2)
    return WL_EINVAL;
  const double xa = 1.0 / (1.0 + sp->a / sp->T_max);
  for (int32_t t = 0; t < sp->n_T; ++t) {
    const int32_t k = sp->n_T - t;
    const double x = k * xa / sp->n_T;
    T[t] = t == 0 ? sp->a : sp->T_max * (1.0 / x - 1.0);
  }
  for (int32_t j = 0; j < sp->n_rho; ++j) {
    const int32_t k = sp->n_rho - j;
    const double x = (double)k / sp->n_rho;
    rho[j] = j == 0 ? 0.0 : sp->rho_max * (1.0 / x - 1.0);
  }
  return WL_OK;
}

int wl_action(wl_ctx* ctx, const wl_action_spec* sp, const wl_field* field, int32_t spin,
              const double* group_sums, int32_t n_groups, int64_t n_loops, int32_t flags,
              const wl_action_out* out) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!sp || !out) return fail(ctx, WL_EINVAL, "spec or out is NULL");
  if (!(sp->m2 > 0.0 && sp->a > 0.0 && sp->T_max > 0.0 && sp->rho_max > 0.0 &&
        isfinite(sp->m2) && isfinite(sp->a) && isfinite(sp->T_max) && isfinite(sp->rho_max)))
    return fail(ctx, WL_EINVAL, "m2, a, T_max and rho_max must be finite and > 0");
  if (sp->n_T < 2 || sp->n_T % 2 || sp->n_rho < 2 || sp->n_rho % 2)
    return fail(ctx, WL_EINVAL, "n_T and n_rho must be even and >= 2");
  if ((int64_t)sp->n_T * sp->n_rho > ((int64_t)1 << 26))
    return fail(ctx, WL_EINVAL, "grid too large");
  wl::FieldArgs fa;
  int rc = check_field(ctx, field, &fa);
  if (rc) return rc;
  if (spin != 0 && spin != 1) return fail(ctx, WL_EINVAL, "spin must be 0 or 1");
  if (n_groups < 1 || n_groups > (1 << 20) || n_loops < n_groups || n_loops % n_groups)
    return fail(ctx, WL_EINVAL, "n_groups must be >= 1 and divide n_loops");
  if (!group_sums) return fail(ctx, WL_EINVAL, "group_sums is NULL");
  if (flags != WL_HOST_PTR && flags != WL_DEVICE_PTR)
    return fail(ctx, WL_EINVAL, "unknown flags %d", flags);
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const int64_t G = n_groups, nr = sp->n_rho, nt = sp->n_T;
  const int64_t sums_n = flags == WL_HOST_PTR ? G * nr * nt : 0;
  const int64_t dens_n = (G + 1) * nr, act_n = G + 1;
  const size_t need = (size_t)(sums_n + dens_n + act_n + 2 * nr + 2) * sizeof(double);
  void* buf = nullptr;
  if (hipMalloc(&buf, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM, "hipMalloc(%zu bytes) for the action failed", need);
  }
  double* d_sums = flags == WL_HOST_PTR ? (double*)buf : (double*)group_sums;
  double* d_dens = (double*)buf + sums_n;
  double* d_act = d_dens + dens_n;
  double* d_dmean = d_act + act_n;
  double* d_derr = d_dmean + nr;
  double* d_am = d_derr + nr;
  hipError_t e = hipSuccess;
  if (flags == WL_HOST_PTR)
    e = hipMemcpyAsync(d_sums, group_sums, sums_n * sizeof(double), hipMemcpyHostToDevice,
                       ctx->stream);
  if (e == hipSuccess)
    e = wl::launch_action(*sp, field->kind, field->eB0, field->lambda, spin, d_sums,
                          n_groups, n_loops, d_dens, d_act, d_dmean, d_derr, d_am,
                          ctx->stream);
  const hipMemcpyKind k =
      flags == WL_HOST_PTR ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  auto put = [&](double* dst, const double* src, int64_t n) {
    if (e == hipSuccess && dst) e = hipMemcpyAsync(dst, src, n * sizeof(double), k, ctx->stream);
  };
  put(out->density, d_dens, G * nr);
  put(out->density_mean, d_dmean, nr);
  put(out->density_err, d_derr, nr);
  put(out->action, d_act, G);
  put(out->action_mean, d_am, 1);
  put(out->action_err, d_am + 1, 1);
  put(out->lcf_density, d_dens + G * nr, nr);
  put(out->lcf_action, d_act + G, 1);
  // the scratch buffer is freed once the work has finished
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_action");
  return WL_OK;
}

}  // extern "C"
