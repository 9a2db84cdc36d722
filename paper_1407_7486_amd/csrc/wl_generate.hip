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

// One workgroup per loop (grid-stride over loops), one coordinate per pass
// (comp 0: x from the cosines, 1: y from the sines): the loop's N FP64
// values sit in LDS (8N bytes).  Threads take the new points of a level;
// a barrier separates the levels.
__global__ __launch_bounds__(256) void k_generate(uint64_t seed, int64_t first_loop,
                                                  int64_t n_loops, int32_t n_ppl,
                                                  int32_t comp, float* __restrict__ out) {
#pragma clang fp contract(off)
  extern __shared__ double v[];
  __shared__ double part[256];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const double two_pi = 6.283185307179586476925286766559;
  const double inv32 = 1.0 / 4294967296.0;
  for (int64_t l = blockIdx.x; l < n_loops; l += gridDim.x) {
    const uint64_t gl = (uint64_t)(first_loop + l);
    if (threadIdx.x == 0) v[0] = 0.0;
    __syncthreads();
    for (int32_t nk = 2; nk <= n_ppl; nk *= 2) {
      const int32_t h = n_ppl / nk;
      const double sigma = 1.0 / sqrt((double)nk);
      for (int32_t qi = threadIdx.x; qi < nk / 2; qi += blockDim.x) {
        const int32_t i = (2 * qi + 1) * h;
        const int32_t a = i - h;
        const int32_t b = (i + h == n_ppl) ? 0 : i + h;
        const int64_t p = (int64_t)(nk / 2 - 1) + qi;  // ordinal of the new point
        uint32_t w[4];
        philox4x32_10((uint32_t)(p >> 1), (uint32_t)gl, (uint32_t)(gl >> 32), 0u, k0, k1, w);
        const int pr = (int)(p & 1);
        const double u1 = ((double)w[2 * pr] + 0.5) * inv32;
        const double u2 = ((double)w[2 * pr + 1] + 0.5) * inv32;
        const double r = sqrt(-2.0 * log(u1));
        const double z = comp == 0 ? r * cos(two_pi * u2) : r * sin(two_pi * u2);
        const double mid = 0.5 * (v[a] + v[b]);
        const double dz = sigma * z;
        v[i] = mid + dz;
      }
      __syncthreads();
    }
    // centre of mass
    double s = 0.0;
    for (int32_t i = threadIdx.x; i < n_ppl; i += blockDim.x) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int32_t w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int32_t)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
      __syncthreads();
    }
    const double mean = part[0] / n_ppl;
    float* o = out + l * n_ppl;
    for (int32_t i = threadIdx.x; i < n_ppl; i += blockDim.x) o[i] = (float)(v[i] - mean);
    __syncthreads();  // v and part are reused by the next loop
  }
}

}  // namespace

hipError_t launch_generate(uint64_t seed, int64_t first_loop, int64_t n_loops, int32_t n_ppl,
                           float* d_x, float* d_y, hipStream_t stream) {
  int64_t blocks = n_loops < 65536 ? n_loops : 65536;
  const size_t lds = (size_t)n_ppl * sizeof(double);
  for (int comp = 0; comp < 2; ++comp) {
    hipLaunchKernelGGL(k_generate, dim3((uint32_t)blocks), dim3(256), lds, stream, seed,
                       first_loop, n_loops, n_ppl, comp, comp == 0 ? d_x : d_y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace wl
