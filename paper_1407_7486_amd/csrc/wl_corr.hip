// Correlation coefficients between grid points over loops or groups
// (Sec. 4.2, Eq. corrcoef) and group sums under a reassignment of the loops
// to groups (Sec. 4.2.3, shuffled groups).
//
// The correlation matrix of n_pts grid points over n_units samples is a
// dense contraction, C = Xc^T Xc with Xc the samples minus their column
// means, so it runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// 128 x 128 output tiles per 256-thread workgroup, the centred samples
// staged through LDS 16 rows at a time, only tiles on or above the diagonal
// (C is symmetric), and the sample range split over workgroups when there
// are too few tiles to fill the chip (partials summed in a fixed order, so
// results are deterministic).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "wl_host.h"

namespace wl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;  // output tile edge
constexpr int kBK = 16;     // samples per LDS stage

// Column sums of rows [r*chunk, (r+1)*chunk) into part[r][p].
__global__ __launch_bounds__(256) void k_col_partial(const double* __restrict__ X,
                                                     int64_t n_units, int32_t n_pts,
                                                     int64_t chunk, double* __restrict__ part) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (p >= n_pts) return;
  const int64_t k0 = r * chunk;
  int64_t k1 = k0 + chunk;
  if (k1 > n_units) k1 = n_units;
  double s = 0.0;
  for (int64_t k = k0; k < k1; ++k) s += X[k * n_pts + p];
  part[r * n_pts + p] = s;
}

__global__ __launch_bounds__(256) void k_col_mean(const double* __restrict__ part, int32_t n_rows,
                                                  int32_t n_pts, int64_t n_units,
                                                  double* __restrict__ mu) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  double s = 0.0;
  for (int32_t r = 0; r < n_rows; ++r) s += part[(int64_t)r * n_pts + p];
  mu[p] = s / (double)n_units;
}

// Tile (bm, bn), bn >= bm, of the upper triangle from its linear index.
__device__ __forceinline__ void tile_of(int32_t t, int32_t n_tiles, int32_t& bm, int32_t& bn) {
  int32_t row = 0, rem = t;
  while (rem >= n_tiles - row) {
    rem -= n_tiles - row;
    ++row;
  }
  bm = row;
  bn = row + rem;
}

// Partial Gram matrix of split s: part[s][m][n] = sum over samples k of
// split s of (X[k][m] - mu[m]) (X[k][n] - mu[n]), for the tiles on or above
// the diagonal.  Wave w of the workgroup owns the 64 x 64 quarter
// (w / 2, w % 2) of the tile: 4 x 4 MFMA blocks of 16 x 16.
// The samples pass through LDS kBK rows at a time in two buffers: while the
// matrix cores work on one stage, the next stage's global loads are in
// flight into registers and land in the other buffer, so one barrier per
// stage remains and the load latency hides behind the MFMA work.  Rows are
// padded by kPad doubles so that the four 16-lane row groups of a wave's
// LDS read fall on different banks.
constexpr int kPad = 16;

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ X,
                                              const double* __restrict__ mu, int64_t n_units,
                                              int32_t n_pts, int32_t n_tiles, int64_t k_chunk,
                                              double* __restrict__ part) {
  __shared__ double As[2][kBK][kTile + kPad];
  __shared__ double Bs[2][kBK][kTile + kPad];
  const int32_t tid = threadIdx.x;
  const int32_t lane = tid % 64, wave = tid / 64;
  const int32_t wm = wave / 2, wn = wave % 2;
  int32_t bm, bn;
  tile_of(blockIdx.x, n_tiles, bm, bn);
  const int32_t s = blockIdx.y;
  const int64_t k_begin = (int64_t)s * k_chunk;
  int64_t k_end = k_begin + k_chunk;
  if (k_end > n_units) k_end = n_units;
  const int32_t m0 = bm * kTile, n0 = bn * kTile;  // tile origin

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // staging: thread t loads column t % 128 of rows t / 128 + 2 j, j < 8, so
  // that a wavefront reads 64 consecutive doubles of one row per load
  const int32_t lc = tid % kTile, lr0 = tid / kTile;
  const int32_t m = m0 + lc, n = n0 + lc;
  const double mu_m = m < n_pts ? mu[m] : 0.0;
  const double mu_n = n < n_pts ? mu[n] : 0.0;
  // loads are unconditional, from a clamped (in-range) address, and the
  // value is masked afterwards: a guarded load would become a branch with
  // its own wait, serialising the stage's loads (diagonal tiles load their
  // columns twice for the same reason)
  const int32_t mc = m < n_pts ? m : n_pts - 1, nc = n < n_pts ? n : n_pts - 1;
  double xa[kBK / 2], xb[kBK / 2];  // raw values of the stage in flight
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < kBK / 2; ++j) {
      const int64_t k = k0 + lr0 + 2 * j;
      const int64_t kc = k < k_end ? k : k_end - 1;
      xa[j] = X[kc * n_pts + mc];
      xb[j] = X[kc * n_pts + nc];
    }
  };
  // centring and masking happen here, after the stage's matrix work, so
  // that nothing waits for the loads before it
  auto stash = [&](int buf, int64_t k0) {
#pragma unroll
    for (int j = 0; j < kBK / 2; ++j) {
      const bool krow = k0 + lr0 + 2 * j < k_end;
      As[buf][lr0 + 2 * j][lc] = (krow && m < n_pts) ? xa[j] - mu_m : 0.0;
      Bs[buf][lr0 + 2 * j][lc] = (krow && n < n_pts) ? xb[j] - mu_n : 0.0;
    }
  };
  const int32_t n_stage = (int32_t)((k_end - k_begin + kBK - 1) / kBK);
  if (n_stage > 0) {
    fetch(k_begin);
    stash(0, k_begin);
  }
  __syncthreads();
  for (int32_t st = 0; st < n_stage; ++st) {
    const int32_t cur = st & 1;
    const bool more = st + 1 < n_stage;
    const int64_t k_next = k_begin + (int64_t)(st + 1) * kBK;
    if (more) fetch(k_next);
    const double(*A)[kTile + kPad] = As[cur];
    const double(*B)[kTile + kPad] = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const int32_t kr = kk + lane / 16, ci = lane % 16;
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = A[kr][wm * 64 + i * 16 + ci];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = B[kr][wn * 64 + j * 16 + ci];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read in the previous stage, which every wave
    // finished before the barrier that ended it
    if (more) stash(cur ^ 1, k_next);
    __syncthreads();
  }
  // D block layout of the f64 16x16x4 instruction: lane l, element r ->
  // row l / 16 + 4 r, column l % 16
  double* P = part + (int64_t)s * n_pts * n_pts;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int32_t om = m0 + wm * 64 + i * 16 + lane / 16 + 4 * r;
        const int32_t on = n0 + wn * 64 + j * 16 + lane % 16;
        if (om < n_pts && on < n_pts) P[(int64_t)om * n_pts + on] = acc[i][j][r];
      }
}

// rho[p][q] from the split partials; every pair reads the entry (min, max)
// of the upper triangle, so rho is exactly symmetric.
__global__ __launch_bounds__(256) void k_corr(const double* __restrict__ part, int32_t n_split,
                                              int32_t n_pts, double* __restrict__ rho) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_pts * n_pts) return;
  const int32_t p = (int32_t)(t / n_pts), q = (int32_t)(t % n_pts);
  const int32_t a = p < q ? p : q, b = p < q ? q : p;
  const int64_t sz = (int64_t)n_pts * n_pts;
  double c = 0.0, da = 0.0, db = 0.0;
  for (int32_t s = 0; s < n_split; ++s) {
    c += part[s * sz + (int64_t)a * n_pts + b];
    da += part[s * sz + (int64_t)a * n_pts + a];
    db += part[s * sz + (int64_t)b * n_pts + b];
  }
  rho[t] = c / (sqrt(da) * sqrt(db));
}

// sums[g][p] = sum of X[perm_p[g*per + j]][p], j < per, perm_p the
// permutation chosen for point p; an index out of range sets *bad and is
// skipped.
__global__ __launch_bounds__(256) void k_regroup(const double* __restrict__ X, int64_t n_units,
                                                 int32_t n_pts, const int64_t* __restrict__ perms,
                                                 int32_t n_perms,
                                                 const int32_t* __restrict__ point_perm,
                                                 int32_t n_groups, double* __restrict__ sums,
                                                 int* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_groups * n_pts) return;
  const int64_t g = t / n_pts;
  const int32_t p = (int32_t)(t % n_pts);
  int32_t which = point_perm ? point_perm[p] : 0;
  if (which < 0 || which >= n_perms) {
    *bad = 1;
    which = 0;
  }
  const int64_t per = n_units / n_groups;
  const int64_t* pm = perms + (int64_t)which * n_units + g * per;
  double s = 0.0;
  for (int64_t j = 0; j < per; ++j) {
    const int64_t u = pm[j];
    if (u < 0 || u >= n_units) {
      *bad = 1;
      continue;
    }
    s += X[u * n_pts + p];
  }
  sums[t] = s;
}

}  // namespace
}  // namespace wl

using namespace wl;

extern "C" {

int wl_correlation(wl_ctx* ctx, const double* values, int64_t n_units, int32_t n_pts,
                   int32_t flags, double* corr) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!values || !corr) return fail(ctx, WL_EINVAL, "values or corr is NULL");
  if (n_units < 2) return fail(ctx, WL_EINVAL, "need at least 2 samples");
  if (n_pts < 1 || n_pts > 16384) return fail(ctx, WL_EINVAL, "n_pts must be in [1, 16384]");
  if (n_units > ((int64_t)1 << 36) / n_pts) return fail(ctx, WL_EINVAL, "too many samples");
  if (flags != WL_HOST_PTR && flags != WL_DEVICE_PTR)
    return fail(ctx, WL_EINVAL, "unknown flags %d", flags);
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const int32_t n_tiles = (n_pts + kTile - 1) / kTile;
  const int32_t tiles = n_tiles * (n_tiles + 1) / 2;
  // split the samples so that ~16 workgroups per CU have work (the last
  // round of a launch is then a small share of it), in chunks of at least
  // 256 samples, with at most 4 GiB of partials
  int64_t n_split = (16 * (int64_t)ctx->num_cu + tiles - 1) / tiles;
  if (n_split > 8) n_split = 8;
  while (n_split > 1 && n_split * (int64_t)n_pts * n_pts * 8 > ((int64_t)4 << 30)) --n_split;
  const int64_t max_split = (n_units + 255) / 256;
  if (n_split > max_split) n_split = max_split;
  if (n_split < 1) n_split = 1;
  int64_t k_chunk = (n_units + n_split - 1) / n_split;
  k_chunk = (k_chunk + kBK - 1) / kBK * kBK;
  n_split = (n_units + k_chunk - 1) / k_chunk;
  const int32_t mean_rows = (int32_t)((n_units + 4095) / 4096 < 256 ? (n_units + 4095) / 4096 : 256);
  const int64_t mean_chunk = (n_units + mean_rows - 1) / mean_rows;
  const int64_t sz = (int64_t)n_pts * n_pts;
  const int64_t vals_n = flags == WL_HOST_PTR ? n_units * n_pts : 0;
  const int64_t out_n = flags == WL_HOST_PTR ? sz : 0;
  const size_t need =
      (size_t)(vals_n + out_n + n_split * sz + (int64_t)mean_rows * n_pts + n_pts) * sizeof(double);
  void* buf = nullptr;
  if (hipMalloc(&buf, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM, "hipMalloc(%zu bytes) for the correlation failed", need);
  }
  double* d_x = flags == WL_HOST_PTR ? (double*)buf : (double*)values;
  double* d_out = flags == WL_HOST_PTR ? (double*)buf + vals_n : corr;
  double* d_part = (double*)buf + vals_n + out_n;
  double* d_mp = d_part + n_split * sz;
  double* d_mu = d_mp + (int64_t)mean_rows * n_pts;
  hipError_t e = hipSuccess;
  if (flags == WL_HOST_PTR)
    e = hipMemcpyAsync(d_x, values, vals_n * sizeof(double), hipMemcpyHostToDevice,
                       ctx->stream);
  const dim3 cb((n_pts + 255) / 256, mean_rows);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_col_partial, cb, dim3(256), 0, ctx->stream, d_x, n_units, n_pts,
                       mean_chunk, d_mp);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_col_mean, dim3((n_pts + 255) / 256), dim3(256), 0, ctx->stream, d_mp,
                       mean_rows, n_pts, n_units, d_mu);
    e = hipGetLastError();
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess && ctx->timing) {
    e = next_events(ctx, &ev0, &ev1);
    if (e == hipSuccess) e = hipEventRecord(ev0, ctx->stream);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gram, dim3(tiles, (uint32_t)n_split), dim3(256), 0, ctx->stream, d_x,
                       d_mu, n_units, n_pts, n_tiles, k_chunk, d_part);
    e = hipGetLastError();
  }
  if (e == hipSuccess && ctx->timing) {
    e = hipEventRecord(ev1, ctx->stream);
    if (e == hipSuccess) ctx->n_timed++;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_corr, dim3((uint32_t)((sz + 255) / 256)), dim3(256), 0, ctx->stream,
                       d_part, (int32_t)n_split, n_pts, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess && flags == WL_HOST_PTR)
    e = hipMemcpyAsync(corr, d_out, sz * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_correlation");
  return WL_OK;
}

int wl_regroup(wl_ctx* ctx, const double* per_unit, int64_t n_units, int32_t n_pts,
               const int64_t* perms, int32_t n_perms, const int32_t* point_perm,
               int32_t n_groups, int32_t flags, double* sums) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!per_unit || !perms || !sums) return fail(ctx, WL_EINVAL, "NULL array");
  if (n_units < 1 || n_pts < 1 || n_perms < 1)
    return fail(ctx, WL_EINVAL, "n_units, n_pts and n_perms must be >= 1");
  if (n_groups < 1 || n_units % n_groups)
    return fail(ctx, WL_EINVAL, "n_groups must be >= 1 and divide n_units");
  if (n_units > ((int64_t)1 << 36) / n_pts || (int64_t)n_perms * n_units > ((int64_t)1 << 32))
    return fail(ctx, WL_EINVAL, "arrays too large");
  if (flags != WL_HOST_PTR && flags != WL_DEVICE_PTR)
    return fail(ctx, WL_EINVAL, "unknown flags %d", flags);
  if (flags == WL_HOST_PTR) {
    // every row of perms must be a permutation of 0 .. n_units-1
    std::vector<char> seen((size_t)n_units);
    for (int32_t w = 0; w < n_perms; ++w) {
      std::fill(seen.begin(), seen.end(), 0);
      for (int64_t j = 0; j < n_units; ++j) {
        const int64_t u = perms[(int64_t)w * n_units + j];
        if (u < 0 || u >= n_units || seen[(size_t)u])
          return fail(ctx, WL_EINVAL, "perms row %d is not a permutation", w);
        seen[(size_t)u] = 1;
      }
    }
    if (point_perm)
      for (int32_t p = 0; p < n_pts; ++p)
        if (point_perm[p] < 0 || point_perm[p] >= n_perms)
          return fail(ctx, WL_EINVAL, "point_perm[%d] out of range", p);
  }
  DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return hip_fail(ctx, g.status, "hipSetDevice");
  const bool host = flags == WL_HOST_PTR;
  const int64_t xn = host ? n_units * n_pts : 0, pn = host ? (int64_t)n_perms * n_units : 0;
  const int64_t qn = host && point_perm ? n_pts : 0, sn = host ? (int64_t)n_groups * n_pts : 0;
  const size_t need = (size_t)(xn + sn) * sizeof(double) + (size_t)pn * sizeof(int64_t) +
                      (size_t)qn * sizeof(int32_t) + 16;
  void* buf = nullptr;
  if (hipMalloc(&buf, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, WL_ENOMEM, "hipMalloc(%zu bytes) for the regrouping failed", need);
  }
  double* d_x = host ? (double*)buf : (double*)per_unit;
  double* d_s = host ? (double*)buf + xn : sums;
  int64_t* d_p = host ? (int64_t*)((double*)buf + xn + sn) : (int64_t*)perms;
  int32_t* d_q = host ? (point_perm ? (int32_t*)(d_p + pn) : nullptr) : (int32_t*)point_perm;
  hipError_t e = hipSuccess;
  if (host) {
    e = hipMemcpyAsync(d_x, per_unit, xn * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_p, perms, pn * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && d_q)
      e = hipMemcpyAsync(d_q, point_perm, qn * sizeof(int32_t), hipMemcpyHostToDevice,
                         ctx->stream);
  }
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_flag, 0, sizeof(int), ctx->stream);
  const int64_t total = (int64_t)n_groups * n_pts;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_regroup, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0,
                       ctx->stream, d_x, n_units, n_pts, d_p, n_perms, d_q, n_groups, d_s,
                       ctx->d_flag);
    e = hipGetLastError();
  }
  int bad = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&bad, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && host)
    e = hipMemcpyAsync(sums, d_s, sn * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(ctx, e, "wl_regroup");
  if (bad) return fail(ctx, WL_EINVAL, "perms or point_perm hold an index out of range");
  return WL_OK;
}

int wl_ensemble_set_groups(wl_ens* ens, int32_t n_groups) {
  if (!ens) return WL_EINVAL;
  wl_ctx* ctx = ens->ctx;
  ctx->err.clear();
  if (n_groups < 1 || ens->n_loops % n_groups)
    return fail(ctx, WL_EINVAL, "n_groups must be >= 1 and divide n_loops");
  ens->n_groups = n_groups;
  return WL_OK;
}

}  // extern "C"
