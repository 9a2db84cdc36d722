// On-device unit-loop generation: d-loops (Sec. 2.1, Loop Generation,
// Eqs. yn2 and ynk) from a counter-based generator, so that an ensemble is
// created where it is used instead of being copied over PCIe.
//
// Random numbers: Philox4x32-10 as published (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), key = the 64-bit
// seed, counter = (block, loop_lo, loop_hi, 0).  Block b gives four words
// w; word w maps to the uniform (w + 0.5) 2^-32, and the pairs (w0, w1),
// (w2, w3) give two standard normals each by Box-Muller:
// r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).  Loop l uses normals
// 0 .. 2(N-1)-1 of its own stream, in the order the recursion consumes
// them: level by level (N_k = 2, 4, ..., N), new points in ascending order,
// x then y.  New point p (counting from 0 over all levels) therefore takes
// the normal pair p: block p/2, word pair p%2, x from the cosine, y from the
// sine.  This is the convention of the repository's seeded input
// generator, so the same (seed, loop) gives the same loop up to last-bit
// differences of the FP64 log / cos / sin implementations.
//
// Recursion, per loop of N = 2^m points: y[0] = 0; at level N_k with stride
// h = N/N_k, point i = q h (q odd) is the midpoint of y[i-h] and
// y[(i+h) mod N] plus a normal of standard deviation 1/sqrt(N_k) (the
// heat-bath weight of Eq. ynk); finally the loop's mean is subtracted
// (common centre of mass at 0).  FP64 throughout, stored as FP32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wl_internal.h"

namespace wl {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1,
                                              uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;  // Weyl key increments
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// One workgroup per loop (grid-stride over loops), both coordinates in one
// pass: the loop's N FP64 x and y values sit in LDS (16N bytes).  At each
// level the threads take the Philox blocks of the level's new points: a
// block feeds the (one or two) new points of that level whose ordinals it
// covers, so that each block, logarithm and square root is computed once
// (only a block straddling two levels is computed once per level).  A
// barrier separates the levels.
__global__ __launch_bounds__(256) void k_generate(uint64_t seed, int64_t first_loop,
                                                  int64_t n_loops, int32_t n_ppl,
                                                  float* __restrict__ out_x,
                                                  float* __restrict__ out_y) {
#pragma clang fp contract(off)
  extern __shared__ double v[];
  double* vx = v;
  double* vy = v + n_ppl;
  __shared__ double part[2][256];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const double two_pi = 6.283185307179586476925286766559;
  const double inv32 = 1.0 / 4294967296.0;
  for (int64_t l = blockIdx.x; l < n_loops; l += gridDim.x) {
    const uint64_t gl = (uint64_t)(first_loop + l);
    if (threadIdx.x == 0) {
      vx[0] = 0.0;
      vy[0] = 0.0;
    }
    __syncthreads();
    for (int32_t nk = 2; nk <= n_ppl; nk *= 2) {
      const int32_t h = n_ppl / nk;
      const double sigma = 1.0 / sqrt((double)nk);
      // ordinals of this level's new points: o0 .. o1
      const int64_t o0 = nk / 2 - 1, o1 = nk - 2;
      for (int64_t bb = (o0 >> 1) + threadIdx.x; bb <= (o1 >> 1); bb += blockDim.x) {
        uint32_t w[4];
        philox4x32_10((uint32_t)bb, (uint32_t)gl, (uint32_t)(gl >> 32), 0u, k0, k1, w);
        for (int pr = 0; pr < 2; ++pr) {
          const int64_t p = 2 * bb + pr;  // ordinal of the new point
          if (p < o0 || p > o1) continue;
          const int32_t qi = (int32_t)(p - o0);
          const int32_t i = (2 * qi + 1) * h;
          const int32_t a = i - h;
          const int32_t b = (i + h == n_ppl) ? 0 : i + h;
          const double u1 = ((double)w[2 * pr] + 0.5) * inv32;
          const double u2 = ((double)w[2 * pr + 1] + 0.5) * inv32;
          const double r = sqrt(-2.0 * log(u1));
          const double zx = r * cos(two_pi * u2);
          const double zy = r * sin(two_pi * u2);
          const double mx = 0.5 * (vx[a] + vx[b]);
          const double my = 0.5 * (vy[a] + vy[b]);
          const double dx = sigma * zx;
          const double dy = sigma * zy;
          vx[i] = mx + dx;
          vy[i] = my + dy;
        }
      }
      __syncthreads();
    }
    // centre of mass
    double sx = 0.0, sy = 0.0;
    for (int32_t i = threadIdx.x; i < n_ppl; i += blockDim.x) {
      sx += vx[i];
      sy += vy[i];
    }
    part[0][threadIdx.x] = sx;
    part[1][threadIdx.x] = sy;
    __syncthreads();
    for (int32_t w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int32_t)threadIdx.x < w) {
        part[0][threadIdx.x] += part[0][threadIdx.x + w];
        part[1][threadIdx.x] += part[1][threadIdx.x + w];
      }
      __syncthreads();
    }
    const double mean_x = part[0][0] / n_ppl, mean_y = part[1][0] / n_ppl;
    float* ox = out_x + l * n_ppl;
    float* oy = out_y + l * n_ppl;
    for (int32_t i = threadIdx.x; i < n_ppl; i += blockDim.x) {
      ox[i] = (float)(vx[i] - mean_x);
      oy[i] = (float)(vy[i] - mean_y);
    }
    __syncthreads();  // v and part are reused by the next loop
  }
}

}  // namespace

hipError_t launch_generate(uint64_t seed, int64_t first_loop, int64_t n_loops, int32_t n_ppl,
                           float* d_x, float* d_y, hipStream_t stream) {
  const int64_t blocks = n_loops < 65536 ? n_loops : 65536;
  const size_t lds = 2 * (size_t)n_ppl * sizeof(double);  // at most 128 KiB (N <= 8192)
  hipError_t e = hipFuncSetAttribute((const void*)k_generate,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_generate, dim3((uint32_t)blocks), dim3(256), lds, stream, seed,
                     first_loop, n_loops, n_ppl, d_x, d_y);
  return hipGetLastError();
}

}  // namespace wl
