/*
 * ORACLE -- test infrastructure only.  Plain, slow, FP64 CPU evaluation of
 * the worldline Wilson-loop average in a cylindrically symmetric magnetic
 * field (Mazur & Heyl, "Parallel Worldline Numerics: Implementation and
 * Error Analysis", arXiv:1407.7486).  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library; the product
 * path never does.  It shares no code with the GPU library.
 *
 * What it computes, step by step in the paper's order and notation:
 *
 *  Unit loops y_i (i = 0..N-1, closed: y_N == y_0) are scaled by sqrt(T)
 *  and shifted to x_cm = (rho_cm, 0)                      (Sec. 2.1, A4)
 *      r_i = (rho_cm + sqrt(T) y_i^x, sqrt(T) y_i^y).
 *
 *  Scalar part (Sec. 3.2.1, Eqs. rhoi..Ci): with the gauge A = A_phi phi^,
 *  the straight segment r_i -> r_{i+1} contributes
 *      (x^i y^{i+1} - y^i x^{i+1}) * int_0^1 g(rho_i^2(t)) dt,
 *      rho_i^2(t) = A_i + 2 B_i t + C_i t^2,
 *      A_i = |r_i|^2, B_i = r_i . (r_{i+1} - r_i), C_i = |r_{i+1} - r_i|^2,
 *  where g(rho^2) = e A_phi(rho) / rho (the paper's F f(rho^2)/rho^2).
 *  Phi = sum over segments; the scalar Wilson loop is cos(Phi) (its real
 *  part: the imaginary part averages to zero by symmetry).
 *
 *  Fermion part (Sec. 3.2.2, Eq. Wfermfpl): cosh(S),
 *      S = e int_0^T B dtau = (T/N) sum_i int_0^1 b(rho_i^2(t)) dt,
 *  with b(rho^2) = e B(rho).
 *
 *  The per-segment t-integrals use n_q-point Gauss-Legendre on [0,1]
 *  (the paper leaves the rule open; n_q = 1 is the midpoint rule).
 *
 *  w = cos(Phi) * (spin ? cosh(S) : 1) per loop and grid point; loops are
 *  split into G contiguous groups (Sec. 4.2.3) and each group's w are
 *  summed in loop order.
 *
 * Fields (e absorbed: eB0 is the central field, lambda the width), each
 * with b = eB and g = e A_phi / rho = e Phi_B(rho) / (2 pi rho^2), where
 * Phi_B(rho) = int_0^rho 2 pi r B(r) dr is the flux inside radius rho
 * (Sec. 3.1, Eq. BWLN and the profile form of A_phi):
 *   CONST    : b = eB0,                     g = eB0 / 2
 *   SECH2    : b = eB0 sech^2(rho/lam),     g = eB0 (u tanh u - ln cosh u)/u^2,
 *              u = rho/lam
 *   GAUSS    : b = eB0 exp(-rho^2/lam^2),   g = eB0 (1 - exp(-v)) / (2 v),
 *              v = rho^2/lam^2
 *   RATIONAL : the paper's validation profile f = rho^2/(lam^2 + rho^2)
 *              (Sec. 6) with F = eB0 lam^2 / 2:
 *              b = 2 F f'(rho^2) = eB0 lam^4/(lam^2+rho^2)^2,
 *              g = F f / rho^2  = eB0 lam^2 / (2 (lam^2 + rho^2))
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { K_CONST = 0, K_SECH2 = 1, K_GAUSS = 2, K_RATIONAL = 3 };

#define MAX_NQ 8

/* ln cosh u for u >= 0 without cancellation: cosh u = 1 + 2 sinh^2(u/2). */
static double ln_cosh(double u) {
  if (u < 20.0) {
    double sh = sinh(0.5 * u);
    return log1p(2.0 * sh * sh);
  }
  return u - M_LN2 + log1p(exp(-2.0 * u));
}

/* e A_phi / rho as a function of rho^2. */
double wlo_field_g(int kind, double eB0, double lam, double r2) {
  switch (kind) {
    case K_CONST:
      return 0.5 * eB0;
    case K_SECH2: {
      double u = sqrt(r2) / lam;
      if (u < 1e-4) /* Taylor: 1/2 - u^2/4 + u^4/9 - ... */
        return eB0 * (0.5 - 0.25 * u * u);
      return eB0 * (u * tanh(u) - ln_cosh(u)) / (u * u);
    }
    case K_GAUSS: {
      double v = r2 / (lam * lam);
      if (v == 0.0) return 0.5 * eB0;
      return eB0 * (-expm1(-v)) / (2.0 * v);
    }
    case K_RATIONAL:
      return eB0 * lam * lam / (2.0 * (lam * lam + r2));
  }
  return NAN;
}

/* e B as a function of rho^2. */
double wlo_field_b(int kind, double eB0, double lam, double r2) {
  switch (kind) {
    case K_CONST:
      return eB0;
    case K_SECH2: {
      double c = cosh(sqrt(r2) / lam);
      return eB0 / (c * c);
    }
    case K_GAUSS:
      return eB0 * exp(-r2 / (lam * lam));
    case K_RATIONAL: {
      double d = lam * lam + r2;
      return eB0 * lam * lam * lam * lam / (d * d);
    }
  }
  return NAN;
}

/* Gauss-Legendre nodes/weights on [0,1]: roots of P_n by Newton's method
 * from the usual cosine guesses (Legendre recurrence for P_n, P_{n-1});
 * weight 2/((1-x^2) P_n'(x)^2), halved for the interval [0,1]. */
static void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x; /* P_0, P_1 */
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;                                   /* P_n     */
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);   /* P_n'    */
}

int wlo_gauss_legendre(int nq, double* t, double* w) {
  if (nq < 1 || nq > MAX_NQ) return -1;
  for (int i = 0; i < nq; ++i) {
    double x = cos(M_PI * (i + 0.75) / (nq + 0.5)), pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(nq, x, &pn, &dp);
      double dx = pn / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    legendre(nq, x, &pn, &dp);
    t[i] = 0.5 * (1.0 + x);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  return 0;
}

/* Phase Phi (radians) and spin exponent S of one loop at one (rho_cm, T).
 * phase_abs (may be NULL) receives sum_i |segment phase|, the size of the
 * terms the phase is summed from (its conditioning: |Phi| can be far
 * smaller when the terms cancel); phase_sq (may be NULL) sum_i (segment
 * phase)^2, whose square root sets the rounding noise of such a sum. */
int wlo_loop_abs(const double* yx, const double* yy, int32_t n, int kind,
                 double eB0, double lam, double rho, double T, int nq,
                 double* phase, double* spin, double* phase_abs, double* phase_sq) {
  double tq[MAX_NQ], wq[MAX_NQ];
  if (n < 2 || wlo_gauss_legendre(nq, tq, wq) != 0) return -1;
  const double s = sqrt(T);
  double phi = 0.0, sb = 0.0, pabs = 0.0, psq = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t j = (i + 1 == n) ? 0 : i + 1; /* closed loop */
    const double xi = rho + s * yx[i], yi = s * yy[i];
    const double xj = rho + s * yx[j], yj = s * yy[j];
    const double A = xi * xi + yi * yi;
    const double B = xi * (xj - xi) + yi * (yj - yi);
    const double C = (xj - xi) * (xj - xi) + (yj - yi) * (yj - yi);
    const double cross = xi * yj - yi * xj;
    double gint = 0.0, bint = 0.0;
    for (int q = 0; q < nq; ++q) {
      const double r2 = A + 2.0 * B * tq[q] + C * tq[q] * tq[q];
      gint += wq[q] * wlo_field_g(kind, eB0, lam, r2);
      bint += wq[q] * wlo_field_b(kind, eB0, lam, r2);
    }
    phi += cross * gint;
    pabs += fabs(cross * gint);
    psq += (cross * gint) * (cross * gint);
    sb += bint;
  }
  *phase = phi;
  *spin = (T / n) * sb;
  if (phase_abs) *phase_abs = pabs;
  if (phase_sq) *phase_sq = psq;
  return 0;
}

int wlo_loop(const double* yx, const double* yy, int32_t n, int kind,
             double eB0, double lam, double rho, double T, int nq,
             double* phase, double* spin) {
  return wlo_loop_abs(yx, yy, n, kind, eB0, lam, rho, T, nq, phase, spin, NULL, NULL);
}

/*
 * Full evaluation over an ensemble.  X, Y: [n_loops][n] FP64 coordinates.
 * Grid point p = j * n_T + k  (rho[j], T[k]).
 * group_sums: [n_groups][n_rho * n_T]  (required)
 * w_out, phase_out, spin_out, phase_abs_out, phase_sq_out:
 *   [n_loops][n_rho * n_T] (each may be NULL)
 * Returns 0, or -1 on an invalid argument, -2 on allocation failure.
 */
int wlo_evaluate(const double* X, const double* Y, int64_t n_loops, int32_t n,
                 int kind, double eB0, double lam, const double* rho,
                 int32_t n_rho, const double* T, int32_t n_T, int spin, int nq,
                 int32_t n_groups, int32_t n_threads, double* group_sums,
                 double* w_out, double* phase_out, double* spin_out,
                 double* phase_abs_out, double* phase_sq_out) {
  if (n < 2 || n_loops < 1 || n_groups < 1 || n_loops % n_groups != 0 ||
      n_rho < 0 || n_T < 0 || nq < 1 || nq > MAX_NQ)
    return -1;
  const int64_t npts = (int64_t)n_rho * n_T;
  double* wbuf = w_out;
  if (!wbuf && npts > 0) {
    wbuf = (double*)malloc(sizeof(double) * (size_t)(n_loops * npts));
    if (!wbuf) return -2;
  }
  /* a thread count for this call only (the process-wide default stays) */
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t l = 0; l < n_loops; ++l) {
    const double* yx = X + l * n;
    const double* yy = Y + l * n;
    for (int32_t a = 0; a < n_rho; ++a) {
      for (int32_t c = 0; c < n_T; ++c) {
        double ph, S, pa, pq;
        wlo_loop_abs(yx, yy, n, kind, eB0, lam, rho[a], T[c], nq, &ph, &S, &pa, &pq);
        const int64_t p = (int64_t)a * n_T + c;
        const double w = cos(ph) * (spin ? cosh(S) : 1.0);
        wbuf[l * npts + p] = w;
        if (phase_out) phase_out[l * npts + p] = ph;
        if (spin_out) spin_out[l * npts + p] = S;
        if (phase_abs_out) phase_abs_out[l * npts + p] = pa;
        if (phase_sq_out) phase_sq_out[l * npts + p] = pq;
      }
    }
  }
  const int64_t per = n_loops / n_groups;
  for (int32_t g = 0; g < n_groups; ++g) {
    for (int64_t p = 0; p < npts; ++p) {
      double acc = 0.0;
      for (int64_t l = g * per; l < (g + 1) * per; ++l) acc += wbuf[l * npts + p];
      group_sums[(int64_t)g * npts + p] = acc;
    }
  }
  if (wbuf != w_out) free(wbuf);
  return 0;
}

int wlo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
