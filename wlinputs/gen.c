/*
 * Seeded synthetic inputs for the worldline Wilson-loop average: unit
 * "d-loop" ensembles (Sec. 2.1, Loop Generation, Eqs. yn2 and ynk).
 *
 * This file produces INPUTS only.  It holds none of the Wilson-loop
 * arithmetic (no field, phase, spin factor or averaging); both the GPU
 * library and the CPU oracle consume what it writes.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed,
 * counter = (block, loop_lo, loop_hi, 0).  Each block yields four 32-bit
 * words; each word u becomes a uniform (u + 0.5) / 2^32 in (0,1), and
 * consecutive uniform pairs (u1, u2) become two standard normals by the
 * Box-Muller transform: r = sqrt(-2 ln u1), z0 = r cos(2 pi u2),
 * z1 = r sin(2 pi u2).  Loop l consumes normals 0 .. 2(N-1)-1 of its own
 * counter stream, so loop l is the same whatever the ensemble size.
 *
 * d-loop recursion (Sec. 2.1, steps 1-5), per loop of N = 2^m points, 2-D
 * (only the two components transverse to a z-directed field enter):
 *   1. y[0] = 0  (the paper's y_N; index N is identified with 0).
 *   2./3. for level k = 1..m, N_k = 2^k, stride h = N / N_k: for every odd
 *      q < N_k the point i = q h is the midpoint of its neighbours
 *      y[i-h], y[(i+h) mod N] plus a Gaussian of variance 1/N_k per
 *      component (the heat-bath weight exp(-(N_k/4) 2 (y - mid)^2)).
 *      Normals are consumed level by level, q ascending, x before y.
 *   5. subtract the loop's mean (common centre of mass at 0).
 * The FP64 loop is then rounded to FP32 (the stored ensemble precision).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One Philox4x32 round: two 32x32->64 products, then the fixed permutation
 * and key mixing of the published definition. */
static inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
  uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

/* Philox4x32-10: ten rounds, the key bumped by the Weyl constants between
 * rounds. */
void wli_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += PHILOX_W0;
      k[1] += PHILOX_W1;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

/* count standard normals of loop `loop` under `seed` (count even). */
void wli_normals(uint64_t seed, int64_t loop, int64_t count, double* z) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const double two_pi = 6.283185307179586476925286766559;
  const double inv32 = 1.0 / 4294967296.0;
  for (int64_t b = 0; 4 * b < count; ++b) {
    uint32_t ctr[4] = {(uint32_t)b, (uint32_t)loop,
                       (uint32_t)((uint64_t)loop >> 32), 0u};
    uint32_t w[4];
    wli_philox4x32_10(ctr, key, w);
    for (int pr = 0; pr < 2; ++pr) {
      double u1 = ((double)w[2 * pr] + 0.5) * inv32;
      double u2 = ((double)w[2 * pr + 1] + 0.5) * inv32;
      double r = sqrt(-2.0 * log(u1));
      int64_t j = 4 * b + 2 * pr;
      if (j < count) z[j] = r * cos(two_pi * u2);
      if (j + 1 < count) z[j + 1] = r * sin(two_pi * u2);
    }
  }
}

/* Build one d-loop (FP64, CM at 0) of n_ppl = 2^m points from the normals
 * z[0 .. 2(n_ppl-1)-1].  x, y: n_ppl doubles each. */
void wli_dloop_from_normals(const double* z, int32_t n_ppl, double* x,
                            double* y) {
  int64_t used = 0;
  x[0] = 0.0;
  y[0] = 0.0;
  for (int32_t nk = 2; nk <= n_ppl; nk *= 2) {
    const int32_t h = n_ppl / nk;
    const double sigma = 1.0 / sqrt((double)nk);
    for (int32_t q = 1; q < nk; q += 2) {
      const int32_t i = q * h;
      const int32_t a = i - h;
      const int32_t b = (i + h) % n_ppl;
      x[i] = 0.5 * (x[a] + x[b]) + sigma * z[used++];
      y[i] = 0.5 * (y[a] + y[b]) + sigma * z[used++];
    }
  }
  double mx = 0.0, my = 0.0;
  for (int32_t i = 0; i < n_ppl; ++i) {
    mx += x[i];
    my += y[i];
  }
  mx /= n_ppl;
  my /= n_ppl;
  for (int32_t i = 0; i < n_ppl; ++i) {
    x[i] -= mx;
    y[i] -= my;
  }
}

static int is_pow2(int32_t n) { return n >= 2 && (n & (n - 1)) == 0; }

/* Loops first_loop .. first_loop+n_loops-1 of the seeded ensemble, FP32,
 * SoA row-major: xs[l * n_ppl + i], ys[l * n_ppl + i].  Returns 0, or -1 on
 * a bad argument / allocation failure. */
int wli_dloop_ensemble_f32(uint64_t seed, int64_t first_loop, int64_t n_loops,
                           int32_t n_ppl, float* xs, float* ys,
                           int32_t n_threads) {
  if (!is_pow2(n_ppl) || n_loops < 0 || first_loop < 0) return -1;
  int failed = 0;
  /* a thread count for this call only (the process-wide default stays) */
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
#pragma omp parallel num_threads(nt)
  {
    double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n_ppl);
    double* x = (double*)malloc(sizeof(double) * (size_t)n_ppl);
    double* y = (double*)malloc(sizeof(double) * (size_t)n_ppl);
    const int ok = (z && x && y);
    if (!ok) {
#pragma omp atomic write
      failed = 1;
    }
    /* every thread reaches the work-sharing loop, even one whose buffers
     * failed to allocate (it then skips its iterations) */
#pragma omp for schedule(static)
    for (int64_t l = 0; l < n_loops; ++l) {
      if (ok) {
        wli_normals(seed, first_loop + l, 2 * (int64_t)(n_ppl - 1), z);
        wli_dloop_from_normals(z, n_ppl, x, y);
        float* xo = xs + (size_t)l * n_ppl;
        float* yo = ys + (size_t)l * n_ppl;
        for (int32_t i = 0; i < n_ppl; ++i) {
          xo[i] = (float)x[i];
          yo[i] = (float)y[i];
        }
      }
    }
    free(z);
    free(x);
    free(y);
  }
  return failed ? -1 : 0;
}
