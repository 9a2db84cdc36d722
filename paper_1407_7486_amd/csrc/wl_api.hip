// Host side of the C ABI declared in include/wl.h: argument checks, device
// buffers, work decomposition and the launches (kernels in wl_kernels.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "wl_host.h"

namespace wl {

int fail(wl_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_fail(wl_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, WL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static int ensure(wl_ctx* ctx, void** p, size_t* have, size_t need, const char* what) {
  if (need <= *have) return WL_OK;
  if (*p) {
    // pending work may still read the old buffer
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM, "hipMalloc(%zu bytes) for %s failed", need, what);
  }
  *have = need;
  return WL_OK;
}

int check_field(wl_ctx* ctx, const wl_field* f, wl::FieldArgs* a) {
  if (!f) return fail(ctx, WL_EINVAL, "field is NULL");
  if (f->kind < WL_CONST || f->kind > WL_RATIONAL)
    return fail(ctx, WL_EINVAL, "unknown field kind %d", f->kind);
  if (f->reserved != 0) return fail(ctx, WL_EINVAL, "field.reserved must be 0");
  if (!isfinite(f->eB0)) return fail(ctx, WL_EINVAL, "field.eB0 not finite");
  const double lam = f->lambda;
  if (f->kind != WL_CONST && !(isfinite(lam) && lam > 0.0))
    return fail(ctx, WL_EINVAL, "field.lambda must be finite and > 0");
  const double l = (f->kind == WL_CONST) ? 1.0 : lam;
  const double log2e = 1.4426950408889634074;
  a->kind = f->kind;
  a->inv_lam_d = 1.0 / l;
  a->inv_lam2_d = 1.0 / (l * l);
  a->lam2_d = l * l;
  a->inv_lam2 = (float)a->inv_lam2_d;
  a->lam2 = (float)a->lam2_d;
  a->lam2_lo = (float)(a->lam2_d - (double)a->lam2);
  a->thr = 0.0f;
  double e2 = 0.0;
  switch (f->kind) {
    case WL_CONST:  // g = eB0/2, b = eB0
      a->cphi = 0.5 * f->eB0;
      a->cspin = f->eB0;
      break;
    case WL_SECH2:  // g = eB0 lam^2 qa, b = eB0 * 4 * E/(1+E)^2
      a->cphi = f->eB0 * l * l;
      a->cspin = 4.0 * f->eB0;
      break;
    case WL_GAUSS:  // g = (eB0 lam^2/2) (1-E)/rho^2, b = eB0 E
      e2 = -log2e / (l * l);
      a->cphi = 0.5 * f->eB0 * l * l;
      a->cspin = f->eB0;
      a->thr = (float)(0.25 * l * l);  // v < 1/4
      break;
    case WL_RATIONAL:  // g = (eB0 lam^2/2) r, b = eB0 lam^4 r^2
      a->cphi = 0.5 * f->eB0 * l * l;
      a->cspin = f->eB0 * l * l * l * l;
      break;
  }
  // FP32 sech^2 works in units scaled by gs = 2 log2(e)/lambda: its qa is
  // divided by ln2 gs^2 and its cross product multiplied by gs^2
  a->cphi32 = f->kind == WL_SECH2 ? a->cphi * 0.69314718055994530942 : a->cphi;
  a->exp2_scale = (float)e2;
  a->exp2_scale_lo = (float)(e2 - (double)a->exp2_scale);
  return WL_OK;
}

int check_grid(wl_ctx* ctx, const double* rho, int32_t n_rho, const double* T,
               int32_t n_T) {
  if (n_rho < 0 || n_T < 0) return fail(ctx, WL_EINVAL, "negative grid size");
  if ((int64_t)n_rho * n_T > (int64_t)INT32_MAX)
    return fail(ctx, WL_EINVAL, "grid has more than 2^31-1 points");
  if ((n_rho > 0 && !rho) || (n_T > 0 && !T))
    return fail(ctx, WL_EINVAL, "grid pointer is NULL");
  for (int32_t j = 0; j < n_rho; ++j)
    if (!(isfinite(rho[j]) && rho[j] >= 0.0))
      return fail(ctx, WL_EINVAL, "rho[%d] must be finite and >= 0", j);
  for (int32_t k = 0; k < n_T; ++k)
    if (!(isfinite(T[k]) && T[k] > 0.0))
      return fail(ctx, WL_EINVAL, "T[%d] must be finite and > 0", k);
  return WL_OK;
}

int check_common(wl_ctx* ctx, const wl_ens* ens, int32_t spin, int32_t precision) {
  if (!ens) return fail(ctx, WL_EINVAL, "ensemble is NULL");
  if (ens->ctx != ctx) return fail(ctx, WL_EINVAL, "ensemble belongs to another context");
  if (spin != 0 && spin != 1) return fail(ctx, WL_EINVAL, "spin must be 0 or 1");
  if (precision < WL_FP32C || precision > WL_FP32K)
    return fail(ctx, WL_EINVAL, "unknown precision %d", precision);
  return WL_OK;
}

int check_not_study(wl_ctx* ctx, int32_t precision) {
  if (precision == WL_FP32K)
    return fail(ctx, WL_EINVAL,
                "WL_FP32K is a precision-study mode of wl_average and the per-loop calls only");
  return WL_OK;
}

wl::Sched make_sched(const wl_ctx* ctx, const wl_ens* e, int32_t n_pts) {
  wl::Sched s{};
  s.loops_per_group = e->n_loops / e->n_groups;
  s.n_chunks = (n_pts + wl::kWave - 1) / wl::kWave;
  // Split each group's loops into sub-ranges until there are wavefronts for
  // ~16 rounds of 8 per SIMD (4 SIMDs per CU): the items have equal cost,
  // and with many short workgroups the hardware dispatcher keeps every SIMD
  // busy to the end (with one or two rounds, the last one runs part-empty).
  // At most 64 sub-ranges, of at least 8 loops each; the partial sums cost
  // G n_sub n_pts doubles.  The rule depends only on the request and the
  // ensemble, so a request is decomposed the same way alone and in a batch.
  const int64_t target = (int64_t)ctx->num_cu * 4 * 8 * 16;
  const int64_t base = (int64_t)e->n_groups * s.n_chunks;
  int64_t n_sub = (target + base - 1) / base;
  if (n_sub > 64) n_sub = 64;
  if (n_sub > s.loops_per_group / 8) n_sub = s.loops_per_group / 8;
  if (n_sub < 1) n_sub = 1;
  s.loops_per_sub = (s.loops_per_group + n_sub - 1) / n_sub;
  // no empty sub-ranges
  n_sub = (s.loops_per_group + s.loops_per_sub - 1) / s.loops_per_sub;
  s.n_sub = (int32_t)n_sub;
  s.n_items = base * n_sub;
  s.n_wg = 0;  // set by the launcher (workgroup size depends on precision)
  s.n_xcd = 8;  // MI355X: 8 XCDs; workgroups are dealt round-robin
  return s;
}

ReqPlan plan_request(const wl_ctx* ctx, const wl_ens* ens, const wl_request& q) {
  ReqPlan p;
  p.n_pts = q.n_rho * q.n_T;
  if (p.n_pts == 0) return p;
  p.s = make_sched(ctx, ens, p.n_pts);
  const int64_t G = ens->n_groups;
  p.in_bytes = sizeof(ReqDesc) + 8 * (size_t)(q.n_rho + q.n_T);
  // group sums, mean, err, scale, fp_err, escalation flags (one byte per
  // point, padded to 8 with the other requests'), the item scale and
  // rounding accumulators, the item partial sums of w when split, the
  // compacted list of flagged points with its count, and the request's
  // row of the FP64 recomputation table, 8 x 8 bytes (with room for the
  // table's final row and the alignments, also for a batch of one)
  const size_t part = (size_t)G * p.s.n_sub * p.n_pts;
  p.res_bytes = 8 * ((size_t)G * p.n_pts + 4 * (size_t)p.n_pts + 2 * part +
                     (p.s.n_sub > 1 ? part : 0)) +
                (size_t)p.n_pts + 8 + 4 * (size_t)p.n_pts + 8 + 2 * 8 * 8 + 32;
  return p;
}

bool build_batch(const wl_ens* ens, const wl_request* const* reqs, const FieldArgs* fa,
                 const ReqPlan* plans, int32_t n, void* h_in, size_t cap_in, void* d_in,
                 void* d_res, size_t cap_res, BatchLayout* lay) {
  const int64_t G = ens->n_groups;
  *lay = BatchLayout();
  int64_t grid_n = 0;
  for (int32_t i = 0; i < n; ++i) {
    lay->items += plans[i].s.n_items;
    lay->sums_n += G * plans[i].n_pts;
    lay->pts_n += plans[i].n_pts;
    lay->acc_n += G * plans[i].s.n_sub * plans[i].n_pts;
    if (plans[i].s.n_sub > 1) lay->part_n += G * plans[i].s.n_sub * plans[i].n_pts;
    grid_n += reqs[i]->n_rho + reqs[i]->n_T;
  }
  const size_t grids_off = kBatchDescOffset + (((size_t)n * sizeof(ReqDesc) + 255) & ~(size_t)255);
  lay->in_bytes = grids_off + 8 * (size_t)grid_n;
  lay->head_bytes = 8 * (size_t)(lay->sums_n + 4 * lay->pts_n) +
                    (((size_t)lay->pts_n + 7) & ~(size_t)7);
  lay->res_bytes = lay->head_bytes + 8 * (size_t)(2 * lay->acc_n + lay->part_n) +
                   4 * (size_t)(lay->pts_n + n) + 8 + 8 * 8 * ((size_t)n + 1);
  if (lay->in_bytes > cap_in || lay->res_bytes > cap_res) return false;
  char* hb = (char*)h_in;
  BatchHeader* hdr = (BatchHeader*)hb;
  hdr->n_reqs = n;
  hdr->total_items = lay->items;
  hdr->total_sums = lay->sums_n;
  hdr->total_pts = lay->pts_n;
  ReqDesc* desc = (ReqDesc*)(hb + kBatchDescOffset);
  double* h_grid = (double*)(hb + grids_off);
  const double* d_grid = (const double*)((const char*)d_in + grids_off);
  // [sums | mean | err | scale | fp_err | flags (bytes) | acc a | acc v | partials]
  double* d_sums = (double*)d_res;
  double* d_scale = d_sums + lay->sums_n + 2 * lay->pts_n;
  double* d_fperr = d_scale + lay->pts_n;
  uint8_t* d_flags = (uint8_t*)(d_fperr + lay->pts_n);
  double* d_acc_a = (double*)((char*)d_res + lay->head_bytes);
  double* d_acc_v = d_acc_a + lay->acc_n;
  double* d_part = d_acc_v + lay->acc_n;
  int32_t* d_list = (int32_t*)(d_part + lay->part_n);  // [pts_n] lists, then [n] counts
  int32_t* d_count = d_list + lay->pts_n;
  int64_t* d_esc_begin = (int64_t*)(((uintptr_t)(d_count + n) + 7) & ~(uintptr_t)7);
  hdr->esc_begin = d_esc_begin;
  int64_t items = 0, sums = 0, pts = 0, part = 0, acc = 0, go = 0;
  for (int32_t i = 0; i < n; ++i) {
    const wl_request& q = *reqs[i];
    const ReqPlan& pl = plans[i];
    ReqDesc e{};
    e.f = fa[i];
    e.rho = d_grid + go;
    e.T = d_grid + go + q.n_rho;
    memcpy(h_grid + go, q.rho, q.n_rho * sizeof(double));
    memcpy(h_grid + go + q.n_rho, q.T, q.n_T * sizeof(double));
    go += q.n_rho + q.n_T;
    e.out = pl.s.n_sub > 1 ? d_part + part : d_sums + sums;
    e.out_a = d_acc_a + acc;
    e.out_v = d_acc_v + acc;
    e.scale = d_scale + pts;
    e.fp_err = d_fperr + pts;
    e.flags = d_flags + pts;
    e.list = d_list + pts;
    e.count = d_count + i;
    e.item_begin = items;
    e.loops_per_sub = pl.s.loops_per_sub;
    e.sums_begin = sums;
    e.pts_begin = pts;
    e.n_sub = pl.s.n_sub;
    e.n_chunks = pl.s.n_chunks;
    e.n_T = q.n_T;
    e.n_pts = pl.n_pts;
    e.spin = q.spin;
    desc[i] = e;
    lay->sums_begin.push_back(sums);
    lay->pts_begin.push_back(pts);
    items += pl.s.n_items;
    sums += G * pl.n_pts;
    pts += pl.n_pts;
    acc += G * pl.s.n_sub * pl.n_pts;
    if (pl.s.n_sub > 1) part += G * pl.s.n_sub * pl.n_pts;
  }
  return true;
}

void scatter_results(const wl_request& q, const BatchLayout& lay, int32_t i,
                     const double* h_res, int64_t G) {
  const int64_t n_pts = (int64_t)q.n_rho * q.n_T;
  const double* per_pt = h_res + lay.sums_n + lay.pts_begin[i];
  if (q.group_sums)
    memcpy(q.group_sums, h_res + lay.sums_begin[i], G * n_pts * sizeof(double));
  if (q.mean) memcpy(q.mean, per_pt, n_pts * sizeof(double));
  if (q.err) memcpy(q.err, per_pt + lay.pts_n, n_pts * sizeof(double));
  if (q.scale) memcpy(q.scale, per_pt + 2 * lay.pts_n, n_pts * sizeof(double));
  if (q.fp_err) memcpy(q.fp_err, per_pt + 3 * lay.pts_n, n_pts * sizeof(double));
  if (q.escalated)
    memcpy(q.escalated,
           (const uint8_t*)(h_res + lay.sums_n + 4 * lay.pts_n) + lay.pts_begin[i], n_pts);
}

// Event pair for the next timed launch (created on first use).
hipError_t next_events(wl_ctx* ctx, hipEvent_t* a, hipEvent_t* b) {
  if (ctx->n_timed == ctx->events.size()) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      return e;
    }
    ctx->events.emplace_back(e0, e1);
  }
  *a = ctx->events[ctx->n_timed].first;
  *b = ctx->events[ctx->n_timed].second;
  return hipSuccess;
}

// FP64 segment array of the ensemble, built on first use (on `stream`, which
// is then synchronized, so the array is complete for every stream once the
// pointer is published).  One lock serialises the builders of all ensembles:
// a server thread and a caller of the same ensemble may both ask.
hipError_t ensure_seg64(const wl_ens* ens, hipStream_t stream) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (ens->d_seg64) return hipSuccess;
  const int64_t nseg = ens->n_loops * ens->n_ppl;
  double4* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, nseg * sizeof(double4));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hipErrorOutOfMemory;
  }
  e = launch_prep64(ens->d_x, ens->d_y, ens->n_loops, ens->n_ppl, d, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(d);
    return e;
  }
  ens->d_seg64 = d;
  return hipSuccess;
}


// Scratch of the allocation-free evaluation (wl_average_async_noalloc):
// one copy per device, reserved when the code object is loaded on it and
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: the device address is obtained once
// per device with hipGetSymbolAddress (noalloc_scratch_ptr) and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[WL_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device, looked up on the
// first call for each device and kept.
static hipError_t noalloc_scratch_ptr(int device, void** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* ptr[kMaxDev] = {};
  static hipError_t status[kMaxDev] = {};
  static bool done[kMaxDev] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!done[device]) {
    void* p = nullptr;
    status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (status[device] != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    ptr[device] = p;
    done[device] = true;
  }
  *out = ptr[device];
  return status[device];
}

}  // namespace wl

using namespace wl;

extern "C" {

const char* wl_version(void) { return "wl 0.1 (gfx950)"; }

const char* wl_strerror(int code) {
  switch (code) {
    case WL_OK: return "ok";
    case WL_EINVAL: return "invalid argument";
    case WL_ENOMEM: return "out of memory";
    case WL_EHIP: return "HIP runtime error";
    case WL_ENODEV: return "no usable gfx950 device";
  }
  return "unknown error code";
}

const char* wl_last_error(const wl_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int wl_create(wl_ctx** out, int device, void* hip_stream) {
  if (!out) return WL_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return WL_ENODEV;
  }
  if (device < 0 || device >= n) return WL_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return WL_ENODEV;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return WL_ENODEV;
  wl_ctx* c = new (std::nothrow) wl_ctx();
  if (!c) return WL_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->num_cu = prop.multiProcessorCount;
  DeviceGuard g(device);
  if (g.status != hipSuccess || hipMalloc((void**)&c->d_flag, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&c->d_counter, kBatchCounters * sizeof(unsigned int)) != hipSuccess) {
    wl_destroy(c);
    return WL_ENOMEM;
  }
  // with the context's device current: the allocation-free entry point's
  // scratch address on this device (a failure is reported by that entry
  // point only)
  c->noalloc_status = noalloc_scratch_ptr(device, &c->d_noalloc);
  *out = c;
  return WL_OK;
}

int wl_destroy(wl_ctx* ctx) {
  if (!ctx) return WL_OK;
  {
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->d_grid) (void)hipFree(ctx->d_grid);
    if (ctx->d_out) (void)hipFree(ctx->d_out);
    if (ctx->d_partial) (void)hipFree(ctx->d_partial);
    if (ctx->d_flag) (void)hipFree(ctx->d_flag);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->d_batch) (void)hipFree(ctx->d_batch);
    for (auto& pr : ctx->events) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  }
  delete ctx;
  return WL_OK;
}

int wl_ensemble_upload(wl_ctx* ctx, const float* y_x, const float* y_y,
                       int64_t n_loops, int32_t n_ppl, int32_t n_groups,
                       int32_t flags, wl_ens** out) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, WL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!y_x || !y_y) return fail(ctx, WL_EINVAL, "coordinate pointer is NULL");
  if (n_loops < 1) return fail(ctx, WL_EINVAL, "n_loops must be >= 1");
  if (n_ppl < 2) return fail(ctx, WL_EINVAL, "n_ppl must be >= 2");
  if (n_groups < 1 || n_loops % n_groups != 0)
    return fail(ctx, WL_EINVAL, "n_groups must be >= 1 and divide n_loops");
  if (flags != WL_HOST_PTR && flags != WL_DEVICE_PTR)
    return fail(ctx, WL_EINVAL, "unknown flags %d", flags);
  if (n_loops > ((int64_t)1 << 40) / n_ppl)
    return fail(ctx, WL_EINVAL, "ensemble too large");
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const int64_t npts = n_loops * n_ppl;
  wl_ens* e = new (std::nothrow) wl_ens();
  if (!e) return fail(ctx, WL_ENOMEM, "host allocation failed");
  e->ctx = ctx;
  e->n_loops = n_loops;
  e->n_ppl = n_ppl;
  e->n_groups = n_groups;
  auto cleanup = [&](int code) {
    if (e->d_x) (void)hipFree(e->d_x);
    if (e->d_y) (void)hipFree(e->d_y);
    if (e->d_seg) (void)hipFree(e->d_seg);
    if (e->d_norm) (void)hipFree(e->d_norm);
    delete e;
    return code;
  };
  if (hipMalloc((void**)&e->d_x, npts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&e->d_y, npts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&e->d_seg, npts * sizeof(float4)) != hipSuccess ||
      hipMalloc((void**)&e->d_norm, n_loops * sizeof(float2)) != hipSuccess) {
    (void)hipGetLastError();
    return cleanup(fail(ctx, WL_ENOMEM, "device allocation of %lld points failed",
                        (long long)npts));
  }
  const hipMemcpyKind kind =
      flags == WL_DEVICE_PTR ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t err = hipMemcpyAsync(e->d_x, y_x, npts * sizeof(float), kind, ctx->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(e->d_y, y_y, npts * sizeof(float), kind, ctx->stream);
  if (err == hipSuccess) err = hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream);
  if (err == hipSuccess)
    err = wl::launch_prep(e->d_x, e->d_y, n_loops, n_ppl, e->d_seg, e->d_norm, ctx->d_flag,
                           ctx->stream);
  int bad = 0;
  if (err == hipSuccess)
    err = hipMemcpyAsync(&bad, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(ctx->stream);
  if (err != hipSuccess) return cleanup(hip_fail(ctx, err, "ensemble upload"));
  if (bad) return cleanup(fail(ctx, WL_EINVAL, "non-finite loop coordinate"));
  *out = e;
  return WL_OK;
}

int wl_ensemble_generate(wl_ctx* ctx, uint64_t seed, int64_t first_loop, int64_t n_loops,
                         int32_t n_ppl, int32_t n_groups, wl_ens** out) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, WL_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_loops < 1) return fail(ctx, WL_EINVAL, "n_loops must be >= 1");
  if (first_loop < 0) return fail(ctx, WL_EINVAL, "first_loop must be >= 0");
  if (n_ppl < 2 || n_ppl > 8192 || (n_ppl & (n_ppl - 1)))
    return fail(ctx, WL_EINVAL, "d-loops need n_ppl a power of two in [2, 8192]");
  if (n_groups < 1 || n_loops % n_groups != 0)
    return fail(ctx, WL_EINVAL, "n_groups must be >= 1 and divide n_loops");
  if (n_loops > ((int64_t)1 << 40) / n_ppl) return fail(ctx, WL_EINVAL, "ensemble too large");
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const int64_t npts = n_loops * n_ppl;
  wl_ens* e = new (std::nothrow) wl_ens();
  if (!e) return fail(ctx, WL_ENOMEM, "host allocation failed");
  e->ctx = ctx;
  e->n_loops = n_loops;
  e->n_ppl = n_ppl;
  e->n_groups = n_groups;
  auto cleanup = [&](int code) {
    if (e->d_x) (void)hipFree(e->d_x);
    if (e->d_y) (void)hipFree(e->d_y);
    if (e->d_seg) (void)hipFree(e->d_seg);
    if (e->d_norm) (void)hipFree(e->d_norm);
    delete e;
    return code;
  };
  if (hipMalloc((void**)&e->d_x, npts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&e->d_y, npts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&e->d_seg, npts * sizeof(float4)) != hipSuccess ||
      hipMalloc((void**)&e->d_norm, n_loops * sizeof(float2)) != hipSuccess) {
    (void)hipGetLastError();
    return cleanup(fail(ctx, WL_ENOMEM, "device allocation of %lld points failed",
                        (long long)npts));
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t err = hipSuccess;
  if (ctx->timing) {
    err = next_events(ctx, &ev0, &ev1);
    if (err == hipSuccess) err = hipEventRecord(ev0, ctx->stream);
  }
  if (err == hipSuccess)
    err = wl::launch_generate(seed, first_loop, n_loops, n_ppl, e->d_x, e->d_y, ctx->stream);
  if (err == hipSuccess && ctx->timing) {
    err = hipEventRecord(ev1, ctx->stream);
    if (err == hipSuccess) ctx->n_timed++;
  }
  if (err == hipSuccess) err = hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream);
  if (err == hipSuccess)
    err = wl::launch_prep(e->d_x, e->d_y, n_loops, n_ppl, e->d_seg, e->d_norm, ctx->d_flag,
                           ctx->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(ctx->stream);
  if (err != hipSuccess) return cleanup(hip_fail(ctx, err, "ensemble generation"));
  *out = e;
  return WL_OK;
}

int wl_ensemble_download(const wl_ens* ens, float* y_x, float* y_y, int64_t loop0,
                         int64_t n_loops) {
  if (!ens) return WL_EINVAL;
  wl_ctx* ctx = ens->ctx;
  ctx->err.clear();
  if (loop0 < 0 || n_loops < 0 || loop0 + n_loops > ens->n_loops)
    return fail(ctx, WL_EINVAL, "loop range [%lld, %lld) outside the ensemble",
                (long long)loop0, (long long)(loop0 + n_loops));
  if (n_loops == 0) return WL_OK;
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const size_t off = (size_t)(loop0 * ens->n_ppl), cnt = (size_t)(n_loops * ens->n_ppl);
  hipError_t e = hipSuccess;
  if (y_x)
    e = hipMemcpyAsync(y_x, ens->d_x + off, cnt * sizeof(float), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && y_y)
    e = hipMemcpyAsync(y_y, ens->d_y + off, cnt * sizeof(float), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_ensemble_download");
  return WL_OK;
}

int wl_ensemble_free(wl_ens* ens) {
  if (!ens) return WL_OK;
  DeviceGuard g(ens->ctx->device);
  if (ens->ctx->stream) (void)hipStreamSynchronize(ens->ctx->stream);
  else (void)hipDeviceSynchronize();
  (void)hipFree(ens->d_x);
  (void)hipFree(ens->d_y);
  (void)hipFree(ens->d_seg);
  (void)hipFree(ens->d_norm);
  if (ens->d_sub) (void)hipFree(ens->d_sub);
  if (ens->d_seg64) (void)hipFree(ens->d_seg64);
  if (ens->d_sub64) (void)hipFree(ens->d_sub64);
  delete ens;
  return WL_OK;
}

int wl_ensemble_info(const wl_ens* ens, int64_t* n_loops, int32_t* n_ppl,
                     int32_t* n_groups) {
  if (!ens) return WL_EINVAL;
  if (n_loops) *n_loops = ens->n_loops;
  if (n_ppl) *n_ppl = ens->n_ppl;
  if (n_groups) *n_groups = ens->n_groups;
  return WL_OK;
}

int wl_set_timing(wl_ctx* ctx, int32_t enable) {
  if (!ctx) return WL_EINVAL;
  ctx->timing = enable != 0;
  ctx->n_timed = 0;
  return WL_OK;
}

static int elapsed(wl_ctx* ctx, size_t i, double* ms) {
  hipError_t e = hipEventSynchronize(ctx->events[i].second);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, ctx->events[i].first, ctx->events[i].second);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
  *ms = f;
  return WL_OK;
}

int wl_last_kernel_ms(wl_ctx* ctx, double* ms) {
  if (!ctx || !ms) return WL_EINVAL;
  ctx->err.clear();
  if (ctx->n_timed == 0) return fail(ctx, WL_EINVAL, "no timed launch recorded");
  DeviceGuard g(ctx->device);
  return elapsed(ctx, ctx->n_timed - 1, ms);
}

int wl_kernel_ms_total(wl_ctx* ctx, double* total_ms, int64_t* count) {
  if (!ctx || !total_ms || !count) return WL_EINVAL;
  ctx->err.clear();
  if (ctx->n_timed == 0) return fail(ctx, WL_EINVAL, "no timed launch recorded");
  DeviceGuard g(ctx->device);
  double tot = 0.0;
  for (size_t i = 0; i < ctx->n_timed; ++i) {
    double ms;
    int rc = elapsed(ctx, i, &ms);
    if (rc) return rc;
    tot += ms;
  }
  *total_ms = tot;
  *count = (int64_t)ctx->n_timed;
  return WL_OK;
}


static int need_seg64(wl_ctx* ctx, const wl_ens* ens) {
  const hipError_t e = wl::ensure_seg64(ens, ctx->stream);
  if (e == hipErrorOutOfMemory)
    return fail(ctx, WL_ENOMEM, "device allocation of the FP64 segments (%lld bytes) failed",
                (long long)(ens->n_loops * ens->n_ppl * (int64_t)sizeof(double4)));
  if (e != hipSuccess) return hip_fail(ctx, e, "FP64 segments");
  return WL_OK;
}

// Device outputs of one evaluation (each may be NULL but sums).
struct DevOut {
  double* sums;   // [G][n_pts]
  double* mean;   // [n_pts]
  double* err;
  double* scale;
  double* fp_err;
  uint8_t* escalated;
};

// Scratch of one evaluation: the item partial sums of w (when a group's
// loops are split), of the scale and rounding accumulators, the FP64
// recomputation flags and the compacted list of flagged points with its
// count.
static size_t flag_bytes(int32_t n_pts) { return ((size_t)n_pts + 7) & ~(size_t)7; }
// The sub-range partial sums of w (when split), the scale and rounding
// accumulators, the scale of each mean (read by the FP64 recomputation,
// also when the caller does not ask for it), one flag byte and one list
// entry per grid point.
static size_t eval_scratch_bytes(const wl::Sched& s, int64_t n_groups, int32_t n_pts) {
  const size_t part = (size_t)n_groups * s.n_sub * n_pts;
  return 8 * part * (s.n_sub > 1 ? 3 : 2) + 8 * (size_t)n_pts + flag_bytes(n_pts) +
         4 * ((size_t)n_pts + 1);
}

// Enqueue one evaluation; grid and outputs are device memory: the main
// kernel, the per-point scale and rounding estimate (and for WL_FP32C the
// FP64 recomputation of the flagged points), the sub-range reduction and
// the statistics.  With `noalloc` the call allocates nothing: the scratch
// is the static array (ctx->d_noalloc), the FP64 segment array must exist
// already, and no timing events are recorded.
static int average_device(wl_ctx* ctx, const wl_ens* ens, const wl::FieldArgs& fa,
                          const double* d_rho, int32_t n_rho, const double* d_T,
                          int32_t n_T, int32_t spin, int32_t precision, const DevOut& o,
                          bool noalloc = false) {
  const int32_t n_pts = n_rho * n_T;
  if (precision == WL_FP64) {
    if (noalloc) {
      if (!ens->d_seg64)
        return fail(ctx, WL_EINVAL,
                    "the ensemble's FP64 segment array does not exist yet (an FP64 "
                    "wl_average or wl_average_async derives it)");
    } else {
      int rc = need_seg64(ctx, ens);
      if (rc) return rc;
    }
  }
  const wl::Sched s = make_sched(ctx, ens, n_pts);
  const size_t need = eval_scratch_bytes(s, ens->n_groups, n_pts);
  void* buf;
  if (noalloc) {
    if (need > WL_NOALLOC_SCRATCH_BYTES)
      return fail(ctx, WL_EINVAL,
                  "the evaluation needs %zu bytes of scratch, above the %zu-byte array of "
                  "the allocation-free evaluation", need, (size_t)WL_NOALLOC_SCRATCH_BYTES);
    buf = ctx->d_noalloc;
  } else {
    int rc = ensure(ctx, &ctx->d_partial, &ctx->partial_bytes, need, "evaluation scratch");
    if (rc) return rc;
    buf = ctx->d_partial;
  }
  const size_t part = (size_t)ens->n_groups * s.n_sub * n_pts;
  double* p_w = s.n_sub > 1 ? (double*)buf : o.sums;
  double* p_a = (double*)buf + (s.n_sub > 1 ? part : 0);
  double* p_v = p_a + part;
  double* scale = o.scale ? o.scale : p_v + part;
  uint8_t* flags = (uint8_t*)(p_v + part + n_pts);
  int32_t* list = (int32_t*)(flags + flag_bytes(n_pts));
  hipError_t e = hipSuccess;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (ctx->timing && !noalloc) {
    e = next_events(ctx, &ev0, &ev1);
    if (e == hipSuccess) e = hipEventRecord(ev0, ctx->stream);
  }
  if (e == hipSuccess)
    e = wl::launch_average(precision, spin, fa, ens->d_seg, ens->d_seg64, ens->d_norm,
                           ens->n_ppl, d_rho, d_T, n_T, n_pts, s, p_w, p_a, p_v, ctx->stream);
  if (e == hipSuccess && ctx->timing && !noalloc) {
    e = hipEventRecord(ev1, ctx->stream);
    if (e == hipSuccess) ctx->n_timed++;
  }
  if (e == hipSuccess)
    e = wl::launch_scale_escalate(precision, spin, fa, ens->d_x, ens->d_y, ens->n_ppl, d_rho,
                                  d_T, n_T, n_pts, s, ens->n_loops, p_a, p_v, scale,
                                  o.fp_err, flags, list, p_w, ctx->stream);
  if (e == hipSuccess && s.n_sub > 1)
    e = wl::launch_reduce_sub(p_w, ens->n_groups, s.n_sub, n_pts, o.sums, ctx->stream);
  if (e == hipSuccess && (o.mean || o.err))
    e = wl::launch_stats(o.sums, ens->n_groups, n_pts, ens->n_loops, o.mean, o.err,
                         ctx->stream);
  if (e == hipSuccess && o.escalated)
    e = hipMemcpyAsync(o.escalated, flags, n_pts, hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  return WL_OK;
}

static int average_impl(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                        const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                        int32_t spin, int32_t precision, int32_t flags, const wl_result* out,
                        bool noalloc) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!out) return fail(ctx, WL_EINVAL, "result is NULL");
  if (flags != WL_HOST_PTR && flags != WL_DEVICE_PTR)
    return fail(ctx, WL_EINVAL, "unknown flags %d", flags);
  int rc = check_common(ctx, ens, spin, precision);
  if (rc) return rc;
  wl::FieldArgs fa;
  if ((rc = check_field(ctx, field, &fa))) return rc;
  if (flags == WL_DEVICE_PTR) {
    if (n_rho < 0 || n_T < 0) return fail(ctx, WL_EINVAL, "negative grid size");
    if ((int64_t)n_rho * n_T > (int64_t)INT32_MAX)
      return fail(ctx, WL_EINVAL, "grid has more than 2^31-1 points");
    if ((int64_t)n_rho * n_T == 0) return WL_OK;
    if (!rho || !T || !out->group_sums)
      return fail(ctx, WL_EINVAL, "device pointer is NULL");
    if (noalloc && !ctx->d_noalloc)
      return hip_fail(ctx, ctx->noalloc_status, "address of the allocation-free scratch");
    DeviceGuard g(ctx->device);
    if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
    const DevOut o{out->group_sums, out->mean, out->err, out->scale, out->fp_err,
                   out->escalated};
    return average_device(ctx, ens, fa, rho, n_rho, T, n_T, spin, precision, o, noalloc);
  }
  if ((rc = check_grid(ctx, rho, n_rho, T, n_T))) return rc;
  const int64_t n_pts = (int64_t)n_rho * n_T;
  if (n_pts == 0) return WL_OK;
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const size_t gbytes = (size_t)(n_rho + n_T) * sizeof(double);
  const size_t sums_n = (size_t)ens->n_groups * n_pts;
  // [group sums | mean | err | scale | fp_err | escalation flags]
  const size_t obytes = (sums_n + 4 * (size_t)n_pts) * sizeof(double) + (size_t)n_pts;
  if ((rc = ensure(ctx, &ctx->d_grid, &ctx->grid_bytes, gbytes, "grid"))) return rc;
  if ((rc = ensure(ctx, &ctx->d_out, &ctx->out_bytes, obytes, "results"))) return rc;
  double* d_rho = (double*)ctx->d_grid;
  double* d_T = d_rho + n_rho;
  DevOut o;
  o.sums = (double*)ctx->d_out;
  o.mean = o.sums + sums_n;
  o.err = o.mean + n_pts;
  o.scale = o.err + n_pts;
  o.fp_err = o.scale + n_pts;
  o.escalated = (uint8_t*)(o.fp_err + n_pts);
  hipError_t e = hipMemcpyAsync(d_rho, rho, n_rho * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_T, T, n_T * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "grid upload");
  if ((rc = average_device(ctx, ens, fa, d_rho, n_rho, d_T, n_T, spin, precision, o)))
    return rc;
  const struct {
    void* host;
    const void* dev;
    size_t bytes;
  } copies[] = {{out->group_sums, o.sums, sums_n * sizeof(double)},
                {out->mean, o.mean, n_pts * sizeof(double)},
                {out->err, o.err, n_pts * sizeof(double)},
                {out->scale, o.scale, n_pts * sizeof(double)},
                {out->fp_err, o.fp_err, n_pts * sizeof(double)},
                {out->escalated, o.escalated, (size_t)n_pts}};
  for (const auto& c : copies)
    if (e == hipSuccess && c.host)
      e = hipMemcpyAsync(c.host, c.dev, c.bytes, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_average");
  return WL_OK;
}

int wl_average_ex(wl_ctx* ctx, const wl_ens* ens, const wl_field* field, const double* rho,
                  int32_t n_rho, const double* T, int32_t n_T, int32_t spin,
                  int32_t precision, int32_t flags, const wl_result* out) {
  return average_impl(ctx, ens, field, rho, n_rho, T, n_T, spin, precision, flags, out,
                      false);
}

int wl_average_async(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                     const double* d_rho, int32_t n_rho, const double* d_T,
                     int32_t n_T, int32_t spin, int32_t precision,
                     double* d_mean, double* d_err, double* d_group_sums) {
  const wl_result r{d_mean, d_err, d_group_sums, nullptr, nullptr, nullptr};
  return average_impl(ctx, ens, field, d_rho, n_rho, d_T, n_T, spin, precision,
                      WL_DEVICE_PTR, &r, false);
}

int wl_average_async_noalloc(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                             const double* d_rho, int32_t n_rho, const double* d_T,
                             int32_t n_T, int32_t spin, int32_t precision,
                             double* d_mean, double* d_err, double* d_group_sums) {
  const wl_result r{d_mean, d_err, d_group_sums, nullptr, nullptr, nullptr};
  return average_impl(ctx, ens, field, d_rho, n_rho, d_T, n_T, spin, precision,
                      WL_DEVICE_PTR, &r, true);
}

int wl_average(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
               const double* rho, int32_t n_rho, const double* T, int32_t n_T,
               int32_t spin, int32_t precision, double* mean, double* err,
               double* group_sums) {
  const wl_result r{mean, err, group_sums, nullptr, nullptr, nullptr};
  return average_impl(ctx, ens, field, rho, n_rho, T, n_T, spin, precision, WL_HOST_PTR, &r,
                      false);
}

int wl_average_batch(wl_ctx* ctx, const wl_ens* ens, const wl_request* reqs,
                     int32_t n_reqs) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (n_reqs < 0 || (n_reqs > 0 && !reqs)) return fail(ctx, WL_EINVAL, "bad request list");
  int rc = check_common(ctx, ens, 0, WL_FP32C);
  if (rc) return rc;
  std::vector<wl::FieldArgs> fa(n_reqs);
  for (int32_t r = 0; r < n_reqs; ++r) {
    const wl_request& q = reqs[r];
    if ((rc = check_common(ctx, ens, q.spin, q.precision)) ||
        (rc = check_not_study(ctx, q.precision)) ||
        (rc = check_field(ctx, &q.field, &fa[r])) ||
        (rc = check_grid(ctx, q.rho, q.n_rho, q.T, q.n_T))) {
      std::string m = ctx->err;
      return fail(ctx, rc, "request %d: %s", r, m.c_str());
    }
  }
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  for (int prec = WL_FP32C; prec <= WL_FP64; ++prec) {
    std::vector<const wl_request*> rq;
    std::vector<wl::FieldArgs> rf;
    std::vector<ReqPlan> pl;
    size_t in_b = kBatchDescOffset + 256, res_b = 0;
    for (int32_t r = 0; r < n_reqs; ++r) {
      if (reqs[r].precision != prec || (int64_t)reqs[r].n_rho * reqs[r].n_T == 0) continue;
      rq.push_back(&reqs[r]);
      rf.push_back(fa[r]);
      pl.push_back(plan_request(ctx, ens, reqs[r]));
      in_b += pl.back().in_bytes;
      res_b += pl.back().res_bytes;
    }
    if (rq.empty()) continue;
    if (prec == WL_FP64 && (rc = need_seg64(ctx, ens))) return rc;
    int64_t items = 0;
    for (const ReqPlan& p : pl) items += p.s.n_items;
    if (items > 0xffffffffll)
      return fail(ctx, WL_EINVAL, "batch of %lld work items is too large", (long long)items);
    in_b = (in_b + 255) & ~(size_t)255;
    if ((rc = ensure(ctx, &ctx->d_batch, &ctx->batch_bytes, in_b + res_b, "batch buffer")))
      return rc;
    void* d_in = ctx->d_batch;
    double* d_res = (double*)((char*)ctx->d_batch + in_b);
    std::vector<char> h_in(in_b);
    wl::BatchLayout lay;
    if (!build_batch(ens, rq.data(), rf.data(), pl.data(), (int32_t)rq.size(), h_in.data(),
                     in_b, d_in, d_res, res_b, &lay))
      return fail(ctx, WL_EINVAL, "internal: batch layout exceeds its buffer");
    const int64_t want_wg = (lay.items + kWavesPerWG - 1) / kWavesPerWG;
    const int64_t max_wg = (int64_t)ctx->num_cu * 8;
    hipError_t e = hipMemcpyAsync(d_in, h_in.data(), lay.in_bytes, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess)
      e = wl::launch_batch(prec, ens->d_seg, ens->d_seg64, ens->d_norm, ens->d_x, ens->d_y,
                           ens->n_ppl, d_in, ens->n_groups, ens->n_loops, ctx->d_counter,
                           d_res, (int32_t)(want_wg < max_wg ? want_wg : max_wg),
                           ctx->stream);
    std::vector<double> h_res(lay.head_bytes / sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_res.data(), d_res, h_res.size() * sizeof(double),
                         hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "wl_average_batch");
    for (size_t i = 0; i < rq.size(); ++i)
      scatter_results(*rq[i], lay, (int32_t)i, h_res.data(), ens->n_groups);
  }
  return WL_OK;
}

// Sub-loop segment array of the discretisation estimate, derived once per
// ensemble on the ctx stream.
static int ensure_sub(wl_ctx* ctx, const wl_ens* ens) {
  if (ens->d_sub) return WL_OK;
  const int64_t npts = ens->n_loops * ens->n_ppl;
  float4* d = nullptr;
  if (hipMalloc((void**)&d, npts * sizeof(float4)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM, "device allocation of the sub-loop segments (%lld bytes) failed",
                (long long)(npts * (int64_t)sizeof(float4)));
  }
  hipError_t e = wl::launch_prep_sub(ens->d_x, ens->d_y, ens->n_loops, ens->n_ppl, d,
                                     ctx->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    return hip_fail(ctx, e, "sub-loop segments");
  }
  ens->d_sub = d;
  return WL_OK;
}

// FP64 sub-loop segment array, derived once per ensemble on the ctx stream.
static int ensure_sub64(wl_ctx* ctx, const wl_ens* ens) {
  if (ens->d_sub64) return WL_OK;
  const int64_t npts = ens->n_loops * ens->n_ppl;
  double4* d = nullptr;
  if (hipMalloc((void**)&d, npts * sizeof(double4)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM,
                "device allocation of the FP64 sub-loop segments (%lld bytes) failed",
                (long long)(npts * (int64_t)sizeof(double4)));
  }
  hipError_t e = wl::launch_prep_sub64(ens->d_x, ens->d_y, ens->n_loops, ens->n_ppl, d,
                                       ctx->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    return hip_fail(ctx, e, "FP64 sub-loop segments");
  }
  ens->d_sub64 = d;
  return WL_OK;
}

static int check_subloops(wl_ctx* ctx, const wl_ens* ens) {
  if (ens->n_ppl % 4 != 0 || ens->n_ppl < 8)
    return fail(ctx, WL_EINVAL, "sub-loops need n_ppl divisible by 4 and >= 8 (have %d)",
                ens->n_ppl);
  return WL_OK;
}

// Per-loop values of the part of each loop that `sl` names (segments of
// `seg` for the FP32 paths, of `seg64` for FP64).
static int per_loop_impl(wl_ctx* ctx, const wl_ens* ens, const wl::FieldArgs& fa,
                         const float4* seg, const double4* seg64, const wl::SubLoop& sl,
                         const double* rho,
                         int32_t n_rho, const double* T, int32_t n_T, int32_t spin,
                         int32_t precision, int64_t loop0, int64_t n_loops, double* phase,
                         double* spin_exp, double* w);

int wl_per_loop(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                int32_t spin, int32_t precision, int64_t loop0, int64_t n_loops,
                double* phase, double* spin_exp, double* w) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  int rc = check_common(ctx, ens, spin, precision);
  if (rc) return rc;
  wl::FieldArgs fa;
  if ((rc = check_field(ctx, field, &fa))) return rc;
  if ((rc = check_grid(ctx, rho, n_rho, T, n_T))) return rc;
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const wl::SubLoop sl{0, ens->n_ppl, 0, 1};
  if (precision == WL_FP64 && (rc = need_seg64(ctx, ens))) return rc;
  return per_loop_impl(ctx, ens, fa, ens->d_seg, ens->d_seg64, sl, rho, n_rho, T, n_T, spin,
                       precision, loop0, n_loops, phase, spin_exp, w);
}

int wl_subloop_per_loop(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                        const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                        int32_t spin, int32_t precision, int32_t subloop, int64_t loop0,
                        int64_t n_loops, double* phase, double* spin_exp, double* w) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  int rc = check_common(ctx, ens, spin, precision);
  if (rc) return rc;
  wl::FieldArgs fa;
  if ((rc = check_field(ctx, field, &fa))) return rc;
  if ((rc = check_grid(ctx, rho, n_rho, T, n_T))) return rc;
  if ((rc = check_subloops(ctx, ens))) return rc;
  const int32_t h = ens->n_ppl / 2, q = ens->n_ppl / 4;
  wl::SubLoop sl;
  switch (subloop) {
    case WL_SUB_CIRCLE: sl = wl::SubLoop{0, h, 0, 2}; break;
    case WL_SUB_SQUARE: sl = wl::SubLoop{h, q, 1, 4}; break;
    case WL_SUB_TRIANGLE: sl = wl::SubLoop{h + q, q, 3, 4}; break;
    default: return fail(ctx, WL_EINVAL, "unknown sub-loop %d", subloop);
  }
  if (loop0 < 0 || n_loops < 0 || loop0 + n_loops > ens->n_loops)
    return fail(ctx, WL_EINVAL, "loop range [%lld, %lld) outside the ensemble",
                (long long)loop0, (long long)(loop0 + n_loops));
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  if ((rc = precision == WL_FP64 ? ensure_sub64(ctx, ens) : ensure_sub(ctx, ens))) return rc;
  return per_loop_impl(ctx, ens, fa, ens->d_sub, ens->d_sub64, sl, rho, n_rho, T, n_T, spin,
                       precision, loop0, n_loops, phase, spin_exp, w);
}

static int per_loop_impl(wl_ctx* ctx, const wl_ens* ens, const wl::FieldArgs& fa,
                         const float4* seg, const double4* seg64, const wl::SubLoop& sl,
                         const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                         int32_t spin, int32_t precision, int64_t loop0, int64_t n_loops,
                         double* phase, double* spin_exp, double* w) {
  int rc;
  if (loop0 < 0 || n_loops < 0 || loop0 + n_loops > ens->n_loops)
    return fail(ctx, WL_EINVAL, "loop range [%lld, %lld) outside the ensemble",
                (long long)loop0, (long long)(loop0 + n_loops));
  const int64_t n_pts = (int64_t)n_rho * n_T;
  if (n_pts == 0 || n_loops == 0) return WL_OK;
  if (n_loops * n_pts > ((int64_t)1 << 27))
    return fail(ctx, WL_EINVAL, "n_loops * grid points above 2^27 in one call");
  const size_t gbytes = (size_t)(n_rho + n_T) * sizeof(double);
  const size_t each = (size_t)(n_loops * n_pts);
  if ((rc = ensure(ctx, &ctx->d_grid, &ctx->grid_bytes, gbytes, "grid"))) return rc;
  if ((rc = ensure(ctx, &ctx->d_out, &ctx->out_bytes, 3 * each * sizeof(double),
                   "per-loop results")))
    return rc;
  double* d_rho = (double*)ctx->d_grid;
  double* d_T = d_rho + n_rho;
  double* d_ph = (double*)ctx->d_out;
  double* d_sp = d_ph + each;
  double* d_w = d_sp + each;
  hipError_t e = hipMemcpyAsync(d_rho, rho, n_rho * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_T, T, n_T * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = wl::launch_per_loop(precision, spin, fa, seg, seg64, ens->d_x, ens->d_y, ens->n_ppl, sl,
                            d_rho, d_T, n_T, (int32_t)n_pts, loop0, n_loops, d_ph, d_sp, d_w,
                            ctx->stream);
  if (e == hipSuccess && phase)
    e = hipMemcpyAsync(phase, d_ph, each * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && spin_exp)
    e = hipMemcpyAsync(spin_exp, d_sp, each * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && w)
    e = hipMemcpyAsync(w, d_w, each * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "per-loop evaluation");
  return WL_OK;
}

int wl_discretisation(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                      const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                      int32_t spin, int32_t precision, int32_t mode, double* mean,
                      double* err, double* delta, double* group_sums) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  int rc = check_common(ctx, ens, spin, precision);
  if (rc) return rc;
  if ((rc = check_not_study(ctx, precision))) return rc;
  wl::FieldArgs fa;
  if ((rc = check_field(ctx, field, &fa))) return rc;
  if ((rc = check_grid(ctx, rho, n_rho, T, n_T))) return rc;
  if ((rc = check_subloops(ctx, ens))) return rc;
  if (mode != WL_DISC_PAPER && mode != WL_DISC_FULL)
    return fail(ctx, WL_EINVAL, "unknown discretisation mode %d", mode);
  const int64_t n_pts = (int64_t)n_rho * n_T;
  if (n_pts == 0) return WL_OK;
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  if ((rc = precision == WL_FP64 ? ensure_sub64(ctx, ens) : ensure_sub(ctx, ens))) return rc;
  if (precision == WL_FP64 && mode == WL_DISC_FULL && (rc = need_seg64(ctx, ens))) return rc;
  const int64_t G = ens->n_groups;
  const size_t gbytes = (size_t)(n_rho + n_T) * sizeof(double);
  const size_t sums_n = 4 * (size_t)G * n_pts;
  const size_t obytes = (sums_n + 9 * (size_t)n_pts) * sizeof(double);
  if ((rc = ensure(ctx, &ctx->d_grid, &ctx->grid_bytes, gbytes, "grid"))) return rc;
  if ((rc = ensure(ctx, &ctx->d_out, &ctx->out_bytes, obytes, "results"))) return rc;
  const wl::Sched s = make_sched(ctx, ens, (int32_t)n_pts);
  double* level_out = nullptr;
  if (s.n_sub > 1) {
    const size_t need = 3 * (size_t)G * s.n_sub * n_pts * sizeof(double);
    if ((rc = ensure(ctx, &ctx->d_partial, &ctx->partial_bytes, need, "partial sums")))
      return rc;
    level_out = (double*)ctx->d_partial;
  }
  double* d_rho = (double*)ctx->d_grid;
  double* d_T = d_rho + n_rho;
  double* d_sums = (double*)ctx->d_out;
  double* d_mean = d_sums + sums_n;
  double* d_err = d_mean + 4 * n_pts;
  double* d_delta = d_err + 4 * n_pts;
  if (!level_out) level_out = d_sums;
  hipError_t e = hipMemcpyAsync(d_rho, rho, n_rho * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_T, T, n_T * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess && ctx->timing) {
    e = next_events(ctx, &ev0, &ev1);
    if (e == hipSuccess) e = hipEventRecord(ev0, ctx->stream);
  }
  if (e == hipSuccess)
    e = wl::launch_disc(precision, spin, fa, ens->d_seg, ens->d_sub, ens->d_seg64,
                        ens->d_sub64, ens->n_ppl, d_rho, d_T, n_T, (int32_t)n_pts, s,
                        mode == WL_DISC_FULL ? 1 : 0, level_out, ctx->stream);
  if (e == hipSuccess && ctx->timing) {
    e = hipEventRecord(ev1, ctx->stream);
    if (e == hipSuccess) ctx->n_timed++;
  }
  if (e == hipSuccess && s.n_sub > 1)
    e = wl::launch_reduce_sub(level_out, 3 * (int32_t)G, s.n_sub, (int32_t)n_pts, d_sums,
                              ctx->stream);
  if (e == hipSuccess)
    e = wl::launch_disc_finish(d_sums, (int32_t)G, (int32_t)n_pts, ens->n_loops, d_mean,
                               d_err, d_delta, ctx->stream);
  if (e == hipSuccess && group_sums)
    e = hipMemcpyAsync(group_sums, d_sums, sums_n * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && mean)
    e = hipMemcpyAsync(mean, d_mean, 4 * n_pts * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && err)
    e = hipMemcpyAsync(err, d_err, 4 * n_pts * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && delta)
    e = hipMemcpyAsync(delta, d_delta, n_pts * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_discretisation");
  return WL_OK;
}

}  // extern "C"
