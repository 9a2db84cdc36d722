// Host-side internals shared by the C ABI (wl_api.hip) and the serving loop
// (wl_server.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/wl.h"
#include "wl_internal.h"

struct wl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  std::string err;
  // scratch reused across calls (grown on demand, freed by wl_destroy)
  void* d_grid = nullptr;
  size_t grid_bytes = 0;
  void* d_out = nullptr;
  size_t out_bytes = 0;
  void* d_partial = nullptr;
  size_t partial_bytes = 0;
  int* d_flag = nullptr;
  void* d_batch = nullptr;  // batched evaluation: descriptors, grids, results
  size_t batch_bytes = 0;
  unsigned int* d_counter = nullptr;  // work counters of persistent launches
  // device address of the allocation-free entry point's static scratch
  // array on this context's device (nullptr if it could not be obtained;
  // noalloc_status then holds the HIP error)
  void* d_noalloc = nullptr;
  hipError_t noalloc_status = hipSuccess;
  // timing of the main kernel: one event pair per launch since timing was
  // enabled (pairs are pooled and reused)
  bool timing = false;
  size_t n_timed = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};

struct wl_ens {
  wl_ctx* ctx = nullptr;
  int64_t n_loops = 0;
  int32_t n_ppl = 0;
  int32_t n_groups = 0;
  float* d_x = nullptr;
  float* d_y = nullptr;
  float4* d_seg = nullptr;
  float2* d_norm = nullptr;  // per loop: sqrt(sum c^2), sqrt(sum d_y^2)
  // sub-loop segment array of the discretisation estimate, derived on first
  // use by an FP32 discretisation or sub-loop call (same size as d_seg)
  mutable float4* d_sub = nullptr;
  // FP64 segment array of whole loops, derived on first use by an FP64
  // evaluation (twice the size of d_seg)
  mutable double4* d_seg64 = nullptr;
  // FP64 sub-loop segment array (the layout of d_sub), built on first use by
  // an FP64 discretisation or sub-loop call
  mutable double4* d_sub64 = nullptr;
};

namespace wl {

int fail(wl_ctx* ctx, int code, const char* fmt, ...);
int hip_fail(wl_ctx* ctx, hipError_t e, const char* what);
int check_field(wl_ctx* ctx, const wl_field* f, FieldArgs* a);
int check_grid(wl_ctx* ctx, const double* rho, int32_t n_rho, const double* T, int32_t n_T);
int check_common(wl_ctx* ctx, const wl_ens* ens, int32_t spin, int32_t precision);
// WL_EINVAL for WL_FP32K, which only wl_average and the per-loop calls offer.
int check_not_study(wl_ctx* ctx, int32_t precision);
Sched make_sched(const wl_ctx* ctx, const wl_ens* e, int32_t n_pts);
// FP64 segment array of an ensemble, built on first use on `stream`
// (thread-safe; hipErrorOutOfMemory when the allocation fails).
hipError_t ensure_seg64(const wl_ens* ens, hipStream_t stream);
// Event pair for the next timed launch of ctx (pooled; created on first use).
hipError_t next_events(wl_ctx* ctx, hipEvent_t* a, hipEvent_t* b);

// Makes the context's device current for the duration of a call and
// restores the caller's device afterwards.
struct DeviceGuard {
  int prev = -1;
  hipError_t status = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    status = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Sizes of one request inside a batch.
struct ReqPlan {
  Sched s;
  int32_t n_pts = 0;
  size_t in_bytes = 0;   // descriptor + grids
  size_t res_bytes = 0;  // group sums, mean, err, sub-range partials
};
ReqPlan plan_request(const wl_ctx* ctx, const wl_ens* ens, const wl_request& q);

// Lays out a batch of n requests (all of one precision, none empty).
// Host staging `h_in` receives [BatchHeader | descriptors @ kBatchDescOffset
// | grids]; the device copy of it lives at d_in.  Results on the device, at
// d_res: the head [group sums | means | errors | scales | rounding
// estimates | escalation flags (one byte per point, padded to 8)], copied
// back to the host, then the item scale and rounding accumulators, the
// sub-range partials, the compacted lists of flagged points and their
// counts.  Returns false if the capacities are exceeded.
struct BatchLayout {
  int64_t items = 0, sums_n = 0, pts_n = 0, part_n = 0, acc_n = 0;
  size_t in_bytes = 0, res_bytes = 0, head_bytes = 0;
  std::vector<int64_t> sums_begin, pts_begin;  // per request
};
bool build_batch(const wl_ens* ens, const wl_request* const* reqs, const FieldArgs* fa,
                 const ReqPlan* plans, int32_t n, void* h_in, size_t cap_in, void* d_in,
                 void* d_res, size_t cap_res, BatchLayout* out);

// Copies request i's results out of the host copy of the result region's
// head (head_bytes).
void scatter_results(const wl_request& q, const BatchLayout& lay, int32_t i,
                     const double* h_res, int64_t n_groups);

}  // namespace wl
