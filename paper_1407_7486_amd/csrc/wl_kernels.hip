// Wilson-loop ensemble average: HIP kernels for gfx950 (MI355X).
//
// Mapping.  One wavefront owns one work item = (loop group g, sub-range of
// the group's loops, 64 consecutive (rho_cm, T) grid points).  Lane j holds
// grid point j of the chunk and walks every segment of every loop of the
// item in order.  The segment data of the loop being walked are the same
// for all 64 lanes, so they arrive through wave-uniform (scalar) loads and
// sit in SGPRs, or (the compensated walks of every field but the sech^2
// spinor one) are copied 64 at a time into a per-wave LDS buffer and read
// back as broadcasts: one fetch of a segment serves 64 (rho, T)
// evaluations, and the loop tile is reused across the whole grid.  A lane's
// per-loop phase and spin sums therefore need no
// wavefront reduction, and its FP64 group-sum accumulator has exactly one
// owner and a fixed loop order (deterministic results).
//
// Arithmetic per segment (Sec. 3.2.1, Eqs. rhoi..Ci with the midpoint rule
// t = 1/2, and Sec. 3.2.2, Eq. Wfermfpl), from the unit midpoint m, the unit
// step d and the unit cross product c of the segment:
//   midpoint (rho_cm + s m_x, s m_y),  rho^2 = (rho_cm + s m_x)^2 + T m_y^2
//   cross = U d_y + R c          (U = rho_cm s, R = s^2 = T, s = sqrt(T))
//   phase += cross * qa(rho^2),  spin += qb(rho^2)
// Forming the midpoint (instead of expanding rho^2 around rho_cm^2) keeps
// rho^2 accurate where a loop centred far out crosses the tube axis.  In the
// compensated FP32 mode rho_cm (and the Gaussian and rational field scales)
// are carried as float pairs: their rounding is an error shared by every
// segment of a loop (a shift of the loop by ~1e-7 rho_cm), which cosh(S)
// would amplify by S.
// with qa, qb the field's phase weight and field strength up to constants
// that the FP64 epilogue applies once per loop:
//   Phi = cphi * sum cross qa,   S = cspin (T/N) sum qb,
//   w = cos(Phi) * cosh(S).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wl_internal.h"
#include "wl_poly.h"

namespace wl {
namespace {

constexpr float kLn2f = 0.69314718055994531f;
constexpr double kLn2 = 0.69314718055994530942;
// sech^2 FP32 path in scaled units: geometry multiplied by
// gs = 2 log2(e)/lambda, so that r2 = (2 u log2 e)^2 (u = rho/lambda)
constexpr double kTwoLog2e = 2.8853900817779268147;
constexpr double kLog2e = 1.4426950408889634074;
constexpr float kSech2ThrS = (float)(0.25 * kTwoLog2e * kTwoLog2e);    // u < 1/2
constexpr float kSech2Vs = (float)(1.0 / (kTwoLog2e * kTwoLog2e));     // r2 -> u^2
constexpr float kSech2Ps = (float)(1.0 / (kLn2 * kTwoLog2e * kTwoLog2e));

enum { kConst = 0, kSech2 = 1, kGauss = 2, kRational = 3 };

// ----------------------------------------------------------- FP32 fields
template <int DEG>
__device__ __forceinline__ float horner_f32(const float (&c)[DEG + 1], float v) {
  float acc = c[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) acc = fmaf(acc, v, c[k]);
  return acc;
}

// acc * v + c as the three-address v_fma_f64.  The compiler's choice for a
// running sum acc + v c is the two-address v_fmac_f64, which is fine; this
// form keeps a loop-invariant addend from being copied before every use.
__device__ __forceinline__ double fma3_f64(double acc, double v, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(v), "v"(c));
  return r;
}

// acc * v + c as the three-address v_fma_f64 with the coefficient c in a
// scalar register pair.  Polynomial coefficients as vector operands are
// loop-invariant values the compiler holds in vector registers across the
// segment walk (two per coefficient: 53 in the FP64 walk's polynomials, 16
// more in the per-loop cosine), which under a register budget are spilled to
// scratch and reloaded for every loop or segment; as scalar operands they
// sit in scalar registers (constant-memory loads, or two s_mov each) and the
// FMA reads them directly.  (The two-address v_fmac_f64 would overwrite its
// addend, so a coefficient addend would first be copied into a vector
// register at every step.)
__device__ __forceinline__ double fma3s_f64(double acc, double v, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(v), "s"(c));
  return r;
}

// Horner with every coefficient in scalar registers, for the per-loop
// epilogue (between segment walks, where any vector register held across
// the walk is spilled).  The first step is c[DEG] v (rounded) + c[DEG-1]:
// an FMA of two constants would need two scalar operands, which a VOP3
// instruction on this chip cannot read.
template <int DEG>
__device__ __forceinline__ double horner_s_f64(const double (&c)[DEG + 1], double v) {
  double t, acc;
  asm("v_mul_f64 %0, %1, %2" : "=v"(t) : "v"(v), "s"(c[DEG]));
  asm("v_add_f64 %0, %1, %2" : "=v"(acc) : "v"(t), "s"(c[DEG - 1]));
#pragma unroll
  for (int k = DEG - 2; k >= 0; --k) acc = fma3s_f64(acc, v, c[k]);
  return acc;
}

// Horner for the FP64 segment walk: the leading coefficient in a vector
// register pair (held across the walk, one pair per polynomial), the
// others as scalar operands, so that the first step stays one FMA.  With
// every coefficient a vector operand the FP64 sech^2 spinor kernel needed
// 128 VGPRs (4 waves per SIMD); in this form it needs 60 (8 waves).
template <int DEG>
__device__ __forceinline__ double horner_sv_f64(const double (&c)[DEG + 1], double v) {
  double acc;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(acc) : "v"(c[DEG]), "v"(v), "s"(c[DEG - 1]));
#pragma unroll
  for (int k = DEG - 2; k >= 0; --k) acc = fma3s_f64(acc, v, c[k]);
  return acc;
}

// cos(2 pi r) for |r| <= 1/2: r = f + j/4 with j the nearest quarter turn
// (f = r - j/4 is exact, |f| <= 1/8), then cos(2 pi f), -sin, -cos or sin
// for j = 0, 1, 2, 3 (mod 4), each from its polynomial in f^2 (relative
// error at FP64 rounding).  NaN in, NaN out.
__device__ __forceinline__ double cos2pi(double r) {
  const double j = rint(4.0 * r);
  const double f = fma(-0.25, j, r);
  const double v = f * f;
  const double c = horner_s_f64<WL_COS2PI_F64_DEG>(WL_COS2PI_F64, v);
  const double s = f * horner_s_f64<WL_SIN2PI_F64_DEG>(WL_SIN2PI_F64, v);
  const int q = (int)j & 3;
  const double m = (q & 1) ? s : c;
  return (q == 1 || q == 2) ? -m : m;
}

// qa: phase weight, qb: spin integrand, as functions of rho^2 (FP32,
// hardware transcendentals: v_exp/v_log are base 2, v_rcp/v_rsq 1 ulp).
// Units (the epilogue constants cphi, cspin restore them):
//   SECH2  qa = g/(eB0 lambda^2 ln2 gs^2), gs = 2 log2(e)/lambda, with r2
//          (and the caller's cross product) in units scaled by gs
//          qb = sech^2(u)/4
//   GAUSS  qa = 2g/(eB0 lambda^2)   qb = b/eB0
//   RATIONAL qa = 1/(lambda^2+rho^2) qb = qa^2
// r2 > 0 (the caller adds 1e-30).
// qe: the scale of qa's rounding error, qa itself except where qa is formed
// as the difference of two larger parts (the far branches of sech^2 and the
// Gaussian, 1/r2 times 1 - hp or 1 - E): there the parts' size 1/r2, since
// their rounding, relative to them, carries over to the difference.
// thr: the near-axis threshold on r2 (sech^2: kSech2ThrS; Gaussian: f.thr),
// passed in a vector register (see loop_sums_f32).
template <int KIND, bool COMP>
__device__ __forceinline__ void field_f32(float r2, const FieldArgs& f, float thr,
                                          float& qa, float& qb, float& qe) {
  if constexpr (KIND == kConst) {
    (void)r2;
    (void)f;
    qa = 1.0f;
    qb = 1.0f;
    qe = 1.0f;
  } else if constexpr (KIND == kSech2) {
    // r2 is in scaled units, r2 = t^2 with t = 2 u log2(e) and u = rho/lambda
    // (the geometry multiplied by gs = 2 log2(e)/lambda).  Then E = exp(-2u)
    // = 2^-t, sech^2 u = 4 E/(1+E)^2, and since
    // u tanh u - ln cosh u = ln2 (1 - log2(1+E) - t E/(1+E)) the phase weight
    // is qa = (1 - log2(1+E) - t E/(1+E)) / r2: g/(eB0 lambda^2) divided by
    // ln2 gs^2.  The cross product's parts are in the same units (gs^2 times
    // the unscaled ones), so gs^2 cancels in the product and the FP32
    // epilogue constant cphi32 carries ln2.  The terms cancel as u -> 0: below
    // u = 1/2 a degree-4 polynomial in u^2 is used; between 1/2 and 1 the
    // cancellation costs at most a factor ~6 (per-segment relative error
    // below 1e-6), and fewer waves carry a near lane than with u < 1.
    const float q = __builtin_amdgcn_rsqf(r2);  // 1/t
    const float t = r2 * q;
    const float E = __builtin_amdgcn_exp2f(-t);
    const float opE = 1.0f + E;
    const float ip = __builtin_amdgcn_rcpf(opE);
    const float Eip = E * ip;
    qb = Eip * ip;
    if (r2 < thr) {
      // an empty volatile asm keeps this a branch that waves with no lane
      // near the axis skip; as a short block the compiler would otherwise
      // issue it for every segment
      asm volatile("");
      const float v = r2 * kSech2Vs;
      qa = horner_f32<WL_Q_SECH2_F32_DEG>(WL_Q_SECH2_F32, v) * kSech2Ps;
      qe = qa;
    } else {
      // qa = (1 - hp) q^2 with hp = log2(1+E) + t E/(1+E), q^2 = 1/r2
      const float hp = fmaf(t, Eip, __builtin_amdgcn_logf(opE));
      const float q2 = q * q;
      qa = fmaf(-hp, q2, q2);
      qe = q2;
    }
  } else if constexpr (KIND == kGauss) {
    // v = rho^2/lambda^2, E = exp(-v); 2 g/eB0 = (1-E)/v (polynomial
    // below v = 1/4, where 1-E cancels by more than a factor 4, kept as a
    // branch that waves with no lane that close skip); b/eB0 = E.
    const float E = __builtin_amdgcn_exp2f(
        COMP ? fmaf(r2, f.exp2_scale, r2 * f.exp2_scale_lo) : r2 * f.exp2_scale);
    qb = E;
    if (r2 < thr) {
      asm volatile("");
      const float v = r2 * f.inv_lam2;
      qa = horner_f32<WL_P_GAUSS_F32_DEG>(WL_P_GAUSS_F32, v) * f.inv_lam2;
      qe = qa;
    } else {
      qe = __builtin_amdgcn_rcpf(r2);
      qa = (1.0f - E) * qe;
    }
  } else {  // kRational
    const float r = __builtin_amdgcn_rcpf(COMP ? (r2 + f.lam2) + f.lam2_lo : r2 + f.lam2);
    qa = r;
    qb = r * r;
    qe = r;
  }
}

// ----------------------------------------------------------- FP64 fields
// Elementary functions of the FP64 path, each to a few ulp (the FP64 path
// answers to 1e-12 relative): hardware estimates refined by Newton steps,
// and polynomials whose coefficients (wl_poly.h) sit in constant memory.

// 1/x for x > 0 normal: the hardware estimate (about 23 correct bits) and
// two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// 1/sqrt(x) for x > 0 normal: the hardware estimate and two Newton steps
// y <- y + y (1/2 - (x/2) y^2).
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  return fma(y, fma(-h * y, y, 0.5), y);
}

// 2^-t for t >= 0: -t = n + f with n = rint(-t), |f| <= 1/2 (exact), a
// degree-11 polynomial for 2^f and the exponent added by ldexp.  t is
// clamped at 4096 first (2^-4096 is 0 in FP64), so that n fits an int and f
// stays in range.
__device__ __forceinline__ double exp2_neg64(double t) {
  const double tc = -fmin(t, 4096.0);
  const double n = rint(tc);
  const double p = horner_sv_f64<WL_EXP2_F64_DEG>(WL_EXP2_F64, tc - n);
  return ldexp(p, (int)n);
}

template <int KIND>
__device__ __forceinline__ void field_f64(double r2, const FieldArgs& f,
                                          double& qa, double& qb) {
  if constexpr (KIND == kConst) {
    (void)r2;
    (void)f;
    qa = 1.0;
    qb = 1.0;
  } else if constexpr (KIND == kSech2) {
    // q = 1/rho, t = 2u log2(e) with u = rho/lambda, E = exp(-2u) = 2^-t;
    // 1/r2 = q^2.  Away from the axis (u >= 1/2, so E <= 1/e) the phase
    // weight is (ln2 - ln(1+E) - 2u E/(1+E)) / r2 with ln(1+E) = E P(E).
    const double q = rsq64(r2);
    const double t = (r2 * q) * (kTwoLog2e * f.inv_lam_d);
    const double E = exp2_neg64(t);
    const double ip = rcp64(1.0 + E);
    const double Eip = E * ip;
    qb = Eip * ip;
    const double v = r2 * f.inv_lam2_d;
    if (v < 0.25) {
      qa = horner_sv_f64<WL_Q_SECH2_F64_DEG>(WL_Q_SECH2_F64, v) * f.inv_lam2_d;
    } else {
      const double L = E * horner_sv_f64<WL_LOG1P_F64_DEG>(WL_LOG1P_F64, E);
      qa = fma(-(t * kLn2), Eip, kLn2 - L) * (q * q);
    }
  } else if constexpr (KIND == kGauss) {
    const double v = r2 * f.inv_lam2_d;
    const double E = exp2_neg64(v * kLog2e);
    qb = E;
    qa = v < 0.5 ? horner_sv_f64<WL_P_GAUSS_F64_DEG>(WL_P_GAUSS_F64, v) * f.inv_lam2_d
                 : (1.0 - E) * rcp64(r2);
  } else {
    const double r = rcp64(r2 + f.lam2_d);
    qa = r;
    qb = r * r;
  }
}

// FP64 per-segment quantities (m_x, m_y^2, d_y, c) of the segment from
// (x0, y0) to (x1, y1): m_x and d_y exact, m_y^2 and c rounded once.
__device__ __forceinline__ double4 seg_quantities64(double x0, double y0, double x1,
                                                   double y1) {
  const double my = 0.5 * (y0 + y1);
  double4 o;
  o.x = 0.5 * (x0 + x1);
  o.y = my * my;
  o.z = y1 - y0;
  o.w = x0 * y1 - y0 * x1;
  return o;
}

// An FP64 segment array read in place.
struct SegArray64 {
  const double4* __restrict__ seg;
  __device__ __forceinline__ double4 operator()(int32_t i) const { return seg[i]; }
};

struct LaneF32 {
  float rho_hi, rho_lo;  // rho_cm = hi + lo
  float s_hi;            // sqrt(T)
  float R, U;            // T, rho_cm sqrt(T)
  // sech^2: the same geometry scaled by gs = 2 log2(e)/lambda, all derived
  // from the rounded scaled sqrt(T) so that the scaled loop is one similar
  // figure (R_s = s_s^2, U_s = rho_s s_s up to one rounding each)
  float rho_s_hi, rho_s_lo, s_s, R_s, U_s;
};

__device__ __forceinline__ LaneF32 lane_consts(double rho, double s, double T,
                                               const FieldArgs& f) {
  LaneF32 c;
  c.rho_hi = (float)rho;
  c.rho_lo = (float)(rho - (double)c.rho_hi);
  c.s_hi = (float)s;
  c.R = (float)T;
  c.U = (float)(rho * s);
  const double gs = kTwoLog2e * f.inv_lam_d;
  c.rho_s_hi = (float)(rho * gs);
  c.rho_s_lo = (float)(rho * gs - (double)c.rho_s_hi);
  c.s_s = (float)(s * gs);
  c.R_s = (float)((double)c.s_s * (double)c.s_s);
  c.U_s = (float)(((double)c.rho_s_hi + (double)c.rho_s_lo) * (double)c.s_s);
  return c;
}

// Phase and spin sums of one loop for this lane's grid point (FP32 path).
// `seg` is wave-uniform.  Returns sum cross*qa and sum qb in FP64.
// The cross product cross_i = R c_i + U d_y,i (R = T, U = rho_cm sqrt(T);
// sech^2: their scaled values) is not formed per segment: the two sums
// sum c_i qa_i and sum d_y,i qa_i are kept apart and combined once per loop
// in FP64, one instruction less per segment.  (Where a loop crosses the axis
// far from its centre the two parts cancel within a segment, so each carries
// a rounding error of the size of the larger part: about twice the phase
// error of the combined product there.)
// Compensated mode: each block of 32 segments (four fetches of 8, not
// unrolled together, which keeps the register count at the 8-segment
// level) is summed plainly in FP32 and the block sums accumulate in FP64, so
// the long sum over the loop carries no error growth with N; plain mode
// sums every term in FP32.
// Staged walk (compensated mode, every field but the sech^2 spinor one):
// each wave copies 64 segments at a time into its own LDS buffer (one
// 16-byte load per lane) and reads them back as broadcasts, one segment
// ahead, so that the segment quantities enter the arithmetic from vector
// registers (two-operand forms and an FMA with a literal) instead of scalar
// ones.  Measured: rational -20%, constant -33%, Gaussian -2 to -5%, sech^2
// scalar -1%, the sech^2 spinor walk +0.6% (it keeps the scalar loads); the
// results are the same bits either way.
// Rounding-error estimate (EST), returned in Q:
//   EST 1  Q ~ sum_i qa_i^2, sampled from the first segment of every fetch
//          of 8 (each sample standing for 8 segments; tail segments counted
//          singly), two FMAs per 8 segments;
//   EST 2  Q = sum_i ((|R c_i| + |U d_y,i|) qe_i)^2 exactly (in the units
//          of A), qe_i the scale of qa_i's rounding (field_f32): the
//          squared size of each term's rounding relative to u, the two
//          parts of the cross product being summed apart.
// Per-wave staging buffers of the FP32 segment walk, one of 64 segments for
// each wave of a workgroup (every kernel that walks segments in FP32 runs
// workgroups of at most 8 waves, fixed by its launch bounds).  One array for
// the module, so that a kernel instantiating several walks holds one copy.
__shared__ float4 g_stage[8][kWave];

template <int KIND, bool SPIN, bool COMP, int EST = 0>
__device__ __forceinline__ void loop_sums_f32(const float4* __restrict__ seg,
                                              int32_t n, const LaneF32& c,
                                              const FieldArgs& f, double& A,
                                              double& B, double& Q) {
  constexpr bool kSpinSum = SPIN && KIND != kConst;
  const float Rf = KIND == kSech2 ? c.R_s : c.R;
  const float Uf = KIND == kSech2 ? c.U_s : c.U;
  struct Acc {
    float c, d, b;  // sum c qa, sum d_y qa, sum qb
  };
  float qs = 0.0f;  // rounding-error estimate accumulator (EST)
  // The near-axis threshold, held in a vector register: a compare reading
  // it from a scalar register (where the compiler keeps a constant) issues
  // in ~4.4 cycles per wave, from a vector register in ~2.5.
  float thr = KIND == kSech2 ? kSech2ThrS : KIND == kGauss ? f.thr : 0.0f;
  asm volatile("" : "+v"(thr));
  // sample: 0 not sampled, 1 a sample standing for 8 segments, 2 a single
  // segment (EST 1, in units of 8 segments)
  auto term = [&](const float4 s, Acc& p, int sample) {  // s = (m_x, m_y^2, d_y, c)
    // squared radius of the midpoint (sech^2: in scaled units)
    float r2;
    if constexpr (KIND == kSech2) {
      const float mx = COMP ? fmaf(c.s_s, s.x, c.rho_s_hi) + c.rho_s_lo
                            : fmaf(c.s_s, s.x, c.rho_s_hi);
      r2 = fmaf(mx, mx, fmaf(c.R_s, s.y, 1e-30f));
    } else if constexpr (KIND != kConst) {
      const float mx = COMP ? fmaf(c.s_hi, s.x, c.rho_hi) + c.rho_lo
                            : fmaf(c.s_hi, s.x, c.rho_hi);
      r2 = fmaf(mx, mx, fmaf(c.R, s.y, 1e-30f));
    } else {
      r2 = 1.0f;
    }
    float qa, qb, qe;
    field_f32<KIND, COMP>(r2, f, thr, qa, qb, qe);
    p.c = fmaf(s.w, qa, p.c);
    p.d = fmaf(s.z, qa, p.d);
    if constexpr (kSpinSum) p.b += qb;
    if constexpr (EST == 1) {
      if (sample == 1) qs = fmaf(qa, qa, qs);
      if (sample == 2) qs = fmaf(qa * 0.125f, qa, qs);
    } else if constexpr (EST == 2) {
      // the cross product's two parts are summed apart, each carrying
      // rounding of its own size
      const float x = (fabsf(Rf * s.w) + fabsf(Uf * s.z)) * qe;
      qs = fmaf(x, x, qs);
    }
  };
  double dc = 0.0, dd = 0.0, db = 0.0;  // compensated mode: FP64 block sums
  auto add_block = [&](const Acc& p) {
    dc += (double)p.c;
    dd += (double)p.d;
    if constexpr (kSpinSum) db += (double)p.b;
  };
  Acc s_ = {0.0f, 0.0f, 0.0f};  // plain mode: FP32 sums
  int32_t i = 0;
  if constexpr (COMP && !(KIND == kSech2 && SPIN)) {
    const int32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int32_t ln = threadIdx.x % kWave;
    float4* buf = g_stage[wv];
    for (; i + 64 <= n; i += 64) {
      // every lane's reads of the previous 64 are issued before the buffer
      // is refilled, and the refill before any read (LDS operations of a
      // wave complete in order)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      buf[ln] = seg[i + ln];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
      for (int half = 0; half < 2; ++half) {
        Acc p = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int quarter = 0; quarter < 4; ++quarter) {
          // the index in a vector register: one address register with
          // immediate offsets, not a copy from a scalar one per read
          int32_t idx = 32 * half + 8 * quarter;
          asm volatile("" : "+v"(idx));
          float4 cur = buf[idx];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const float4 nxt = buf[idx + (k < 7 ? k + 1 : k)];
            term(cur, p, k == 0 ? 1 : 0);
            // accumulate here: left to itself the compiler defers the eight
            // segments' accumulations to the end, holding their operands
            asm volatile("" : "+v"(p.c), "+v"(p.d), "+v"(p.b));
            cur = nxt;
          }
        }
        add_block(p);
      }
    }
  }
  if constexpr (COMP) {
    for (; i + 32 <= n; i += 32) {
      Acc p = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
      for (int quarter = 0; quarter < 4; ++quarter) {
        float4 sv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sv[k] = seg[i + 8 * quarter + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) term(sv[k], p, k == 0 ? 1 : 0);
      }
      add_block(p);
    }
  }
  for (; i + 8 <= n; i += 8) {
    // fetch the block's 8 segments up front so that one wait covers them
    float4 sv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) sv[k] = seg[i + k];
    if constexpr (COMP) {
      Acc p = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < 8; ++k) term(sv[k], p, k == 0 ? 1 : 0);
      add_block(p);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) term(sv[k], s_, k == 0 ? 1 : 0);
    }
  }
  if (i < n) {
    Acc p = {0.0f, 0.0f, 0.0f};
    for (; i < n; ++i) term(seg[i], p, 2);
    if constexpr (COMP) {
      add_block(p);
    } else {
      s_.c += p.c;
      s_.d += p.d;
      s_.b += p.b;
    }
  }
  if constexpr (!COMP) {
    dc = s_.c;
    dd = s_.d;
    db = s_.b;
  }
  const double R = Rf;
  const double U = Uf;
  A = R * dc + U * dd;
  B = kSpinSum ? db : (double)n;
  Q = EST == 1 ? 8.0 * (double)qs : (double)qs;
}

// FP32 walk with Kahan-compensated sums (WL_FP32K, a precision-study mode
// in place of the block sums of the compensated mode): the geometry of the
// compensated walk, and each of the three sums (c qa, d_y qa, qb) carried
// in FP32 with its running compensation e (y = x - e, t = s + y,
// e = (t - s) - y, s = t), returned in FP64 as s - e and combined as
// there.  Q is the EST 1 estimate of loop_sums_f32.
template <int KIND, bool SPIN>
__device__ __forceinline__ void loop_sums_f32k(const float4* __restrict__ seg, int32_t n,
                                               const LaneF32& c, const FieldArgs& f,
                                               double& A, double& B, double& Q) {
  constexpr bool kSpinSum = SPIN && KIND != kConst;
  const float Rf = KIND == kSech2 ? c.R_s : c.R;
  const float Uf = KIND == kSech2 ? c.U_s : c.U;
  float thr = KIND == kSech2 ? kSech2ThrS : KIND == kGauss ? f.thr : 0.0f;
  asm volatile("" : "+v"(thr));
  float sc = 0.0f, ec = 0.0f, sd = 0.0f, ed = 0.0f, sb = 0.0f, eb = 0.0f, qs = 0.0f;
  auto kadd = [](float& sum, float& comp, float x) {
    const float y = x - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  };
  // sample: as in loop_sums_f32's EST 1 (units of 8 segments)
  auto term = [&](const float4 s4, int sample) {
    float r2;
    if constexpr (KIND == kSech2) {
      const float mx = fmaf(c.s_s, s4.x, c.rho_s_hi) + c.rho_s_lo;
      r2 = fmaf(mx, mx, fmaf(c.R_s, s4.y, 1e-30f));
    } else if constexpr (KIND != kConst) {
      const float mx = fmaf(c.s_hi, s4.x, c.rho_hi) + c.rho_lo;
      r2 = fmaf(mx, mx, fmaf(c.R, s4.y, 1e-30f));
    } else {
      r2 = 1.0f;
    }
    float qa, qb, qe;
    field_f32<KIND, true>(r2, f, thr, qa, qb, qe);
    kadd(sc, ec, s4.w * qa);
    kadd(sd, ed, s4.z * qa);
    if constexpr (kSpinSum) kadd(sb, eb, qb);
    if (sample == 1) qs = fmaf(qa, qa, qs);
    if (sample == 2) qs = fmaf(qa * 0.125f, qa, qs);
  };
  int32_t i = 0;
  for (; i + 8 <= n; i += 8) {
    float4 sv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) sv[k] = seg[i + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) term(sv[k], k == 0 ? 1 : 0);
  }
  for (; i < n; ++i) term(seg[i], 2);
  const double dc = (double)sc - (double)ec;
  const double dd = (double)sd - (double)ed;
  const double db = (double)sb - (double)eb;
  const double R = Rf;
  const double U = Uf;
  A = R * dc + U * dd;
  B = kSpinSum ? db : (double)n;
  Q = 8.0 * (double)qs;
}

// FP64 path over FP64 segment quantities (m_x, m_y^2, d_y, c) of whole
// loops or sub-loops, each formed from the FP32 points (exact but for one
// rounding of m_y^2 and c) and read from an array: the midpoint's radius
// from m_x and m_y^2, and the
// cross product's two parts summed apart as in the FP32 path,
// cross = s^2 c + rho s d_y.  With EST, Q = sum_i qa_i^2.  `fetch` returns
// segment i's quantities (SegArray64).
template <int KIND, bool SPIN, bool EST, class Fetch>
__device__ __forceinline__ void loop_sums_f64(const Fetch& fetch, int32_t n, double rho,
                                              double s, const FieldArgs& f, double& A,
                                              double& B, double& Q) {
  constexpr bool kSpinSum = SPIN && KIND != kConst;
  const double s2 = s * s;
  double ac = 0.0, ad = 0.0, b = 0.0, q2 = 0.0;
  double4 qn = fetch(0);
  for (int32_t i = 0; i < n; ++i) {
    // the next segment's load is in flight while this one is evaluated
    const double4 q = qn;
    qn = fetch(i + 1 < n ? i + 1 : i);
    const double mx = fma(s, q.x, rho);
    double qa, qb;
    field_f64<KIND>(fma(mx, mx, fma(s2, q.y, 1e-300)), f, qa, qb);
    ac = fma(q.w, qa, ac);
    ad = fma(q.z, qa, ad);
    if constexpr (kSpinSum) b += qb;
    if constexpr (EST) q2 = fma3_f64(qa, qa, q2);
  }
  A = s2 * ac + (rho * s) * ad;
  B = kSpinSum ? b : (double)n;
  Q = q2;
}

// The FP64 sums of a (sub-)loop formed from its raw FP32 points: the
// points first, first + stride, first + 2 stride, ... (indices mod N, m
// segments), so {0, 1} is the whole loop and {0, 2}, {1, 4}, {3, 4} its
// circle, square and triangle sub-loops.  Each segment's quantities are
// those of the FP64 segment arrays (seg_quantities64) and the sums are
// formed as loop_sums_f64 forms them, so the results equal the FP64 path's
// bit for bit.  The points are wave-uniform: they arrive by scalar loads,
// one point ahead, and only the segment in hand occupies vector registers.
template <int KIND, bool SPIN>
__device__ __forceinline__ void loop_sums_f64raw(const float* __restrict__ x,
                                                 const float* __restrict__ y, int32_t n_ppl,
                                                 int32_t first, int32_t stride, int32_t m,
                                                 double rho, double s, const FieldArgs& f,
                                                 double& A, double& B) {
  constexpr bool kSpinSum = SPIN && KIND != kConst;
  const double s2 = s * s;
  double ac = 0.0, ad = 0.0, b = 0.0;
  int32_t a = first;
  float x0 = x[a], y0 = y[a];
  int32_t nb = a + stride;
  if (nb >= n_ppl) nb -= n_ppl;
  float x1 = x[nb], y1 = y[nb];
  for (int32_t j = 0; j < m; ++j) {
    // the point after next is loaded while this segment is evaluated
    int32_t nn = nb + stride;
    if (nn >= n_ppl) nn -= n_ppl;
    const float x2 = x[nn], y2 = y[nn];
    const double4 q = seg_quantities64(x0, y0, x1, y1);
    const double mx = fma(s, q.x, rho);
    double qa, qb;
    field_f64<KIND>(fma(mx, mx, fma(s2, q.y, 1e-300)), f, qa, qb);
    ac = fma(q.w, qa, ac);
    ad = fma(q.z, qa, ad);
    if constexpr (kSpinSum) b += qb;
    x0 = x1;
    y0 = y1;
    x1 = x2;
    y1 = y2;
    nb = nn;
  }
  A = s2 * ac + (rho * s) * ad;
  B = kSpinSum ? b : (double)m;
}

template <int KIND, bool SPIN>
__device__ __forceinline__ void loop_sums_f64seg(const double4* __restrict__ seg, int32_t n,
                                                 double rho, double s, const FieldArgs& f,
                                                 double& A, double& B) {
  double Q;
  loop_sums_f64<KIND, SPIN, false>(SegArray64{seg}, n, rho, s, f, A, B, Q);
}

// Per-loop epilogue in FP64: phase, spin exponent and w.  The phase is
// reduced in revolutions (cos(Phi) = cos(2 pi frac(Phi/2pi))).  The FP32
// paths take cosh from the hardware exp2 of the fractional part of
// S log2(e), scaled by the integer part in FP64 (relative error ~1e-7, no
// overflow below FP64's range).  The FP64 path forms e^|S| = 2^t with
// t = |S| log2(e) carried as t_hi + t_lo (the product's rounding, from an
// FMA, and log2(e)'s own tail), n = rint(t_hi), 2^(t_hi - n) from the
// exp2 polynomial of the segment walk with its coefficients as scalar
// operands, and 2^t_lo as 1 + t_lo ln 2; e^-|S| by the Newton-refined
// reciprocal.  A few ulp; beyond |S| = 709.78 e^|S| is inf (t_hi is held
// below 1100 so that n fits an int), and NaN stays NaN.  (The library exp
// held its coefficients in vector registers that were spilled and
// reloaded for every loop.)
constexpr double kLog2eLo = 2.0355273740931033e-17;  // log2(e) - kLog2e

template <int PREC>
__device__ __forceinline__ double cosh_spin(double S) {
  if constexpr (PREC == 2) {
    const double a = fabs(S);
    const double th = a * kLog2e;
    const double tl = fma(a, kLog2e, -th) + a * kLog2eLo;
    const double tc = th > 1100.0 ? 1100.0 : th;
    const double n = rint(tc);
    const double p0 = horner_s_f64<WL_EXP2_F64_DEG>(WL_EXP2_F64, tc - n);
    const double p = fma(p0 * tl, kLn2, p0);
    const int ni = (int)n;
    return 0.5 * (ldexp(p, ni) + ldexp(rcp64(p), -ni));
  } else {
    const double t = fabs(S) * 1.4426950408889634074;  // |S| log2(e)
    const double k = floor(t);
    const float p = __builtin_amdgcn_exp2f((float)(t - k));  // 2^frac in [1,2)
    const int ki = (int)fminf((float)k, 2000.0f);
    return 0.5 * (ldexp((double)p, ki) + ldexp(1.0 / (double)p, -ki));
  }
}

// The factors of w = cos(phi) cosh(S): cw = cos(phi) (the phase reduced in
// revolutions) and ch = cosh(S) (1 for scalars).
template <bool SPIN, int PREC>
__device__ __forceinline__ void wparts(double phi, double S, double& cw, double& ch) {
  const double rev = phi * 0.15915494309189533577;
  cw = cos2pi(rev - rint(rev));
  ch = SPIN ? cosh_spin<PREC>(S) : 1.0;
}

// w = cw ch as a rounded product, never fused into a caller's sum: every
// kernel that adds w to a sum then gets the same bits.
template <bool SPIN>
__device__ __forceinline__ double wprod(double cw, double ch) {
  if constexpr (!SPIN) {
    return cw;
  } else {
#pragma clang fp contract(off)
    return cw * ch;
  }
}

// w = cos(phi) (scalar) or cos(phi) cosh(S) (spinor).
template <bool SPIN, int PREC>
__device__ __forceinline__ double wval(double phi, double S) {
  double cw, ch;
  wparts<SPIN, PREC>(phi, S, cw, ch);
  return wprod<SPIN>(cw, ch);
}

// phi = cphi A, S = cspin (T/n) B for a loop of n points, and the factors
// of its w.
template <bool SPIN, int PREC>
__device__ __forceinline__ void epilogue_parts(double A, double B, double T, int32_t n,
                                               const FieldArgs& f, double& phi, double& S,
                                               double& cw, double& ch) {
  phi = (PREC == 2 ? f.cphi : f.cphi32) * A;
  S = SPIN ? f.cspin * (T / n) * B : 0.0;
  wparts<SPIN, PREC>(phi, S, cw, ch);
}

template <bool SPIN, int PREC>
__device__ __forceinline__ double epilogue(double A, double B, double T,
                                           int32_t n, const FieldArgs& f,
                                           double& phi, double& S) {
  double cw, ch;
  epilogue_parts<SPIN, PREC>(A, B, T, n, f, phi, S, cw, ch);
  return wprod<SPIN>(cw, ch);
}

// ------------------------------------------------------ rounding estimate
// The FP32 phase of a loop is a sum of n segment terms t_i = cphi cross_i
// qa_i, each carrying independent roundings of a few units u = 2^-24 (the
// stored segment quantities, the midpoint radius, the field evaluation, the
// products and block sums), so its error is of order u sqrt(sum t_i^2); where
// the terms cancel (a loop far off axis in a wide tube, |Phi| << sum |t_i|)
// that exceeds the phase tolerance.  Measured (CPU emulation of this
// arithmetic, and the GPU against the FP64 oracle) the error stays below
// 18 u sqrt(sum t_i^2) on the stress fields; kPhaseK doubles that.
constexpr double kPhaseK = 32.0;
constexpr double kU32 = 5.9604644775390625e-8;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
// Error allowance of a mean for the roundings shared by every loop at a grid
// point (the lane's T and rho_cm constants, smooth errors of the field
// evaluation): they shift all loops alike, so the mean moves like a small
// change of T or of the field, in units of the scale M_S.
constexpr double kSysK = 8.0;

// sqrt(sum_i t_i^2) of one loop from the sampled sum Q ~ sum_i qa_i^2 and
// the loop's norms nc = sqrt(sum c_i^2), nd = sqrt(sum d_y,i^2) (R, U, cphi
// in the units of the path that produced Q): sum (R c_i + U d_i)^2 qa_i^2 is
// taken as (Q/n) (R nc + U nd)^2, i.e. qa_i uncorrelated with the step.
__device__ __forceinline__ double phase_l2(double Q, int32_t n, double R, double U,
                                           float2 nrm, double cphi) {
  return fabs(cphi) * sqrt(Q / (double)n) * (R * (double)nrm.x + U * (double)nrm.y);
}

// Per-loop contributions to the scale and rounding accumulators of a mean:
//   a += |w| max(1, S)                       (the scale M_S, times N_l)
//   v += (sin(phi) cosh(S) l2)^2             (the random rounding of the
//                                              mean, times N_l^2 / (K u)^2)
// (cosh(S) l2 clamped at 1e150 so that v stays finite).
__device__ __forceinline__ void loop_scale(double w, double S, double cw, double ch,
                                           double l2, double& a, double& v) {
  a += fabs(w) * fmax(1.0, S);
  const double x = fmin(ch * l2, 1e150);
  v += fmax(0.0, 1.0 - cw * cw) * (x * x);
}

// The three levels of the discretisation estimate (Sec. 4.1) from the sums
// of the circle (points 0, 2, 4, ...; h = N/2 of them), square (1, 5, 9,
// ...) and triangle (3, 7, 11, ...) sub-loops (q = N/4 points each).  The
// N/2 level is the circle's w.  Paper mode combines the sub-loop phases
// (and spin exponents) as c/2 + s/4 + t/4 for the N level and (s + t)/2 for
// the N/4 level; full mode averages the square and triangle w for the N/4
// level and leaves the N level to the caller (the whole loop).
template <bool SPIN, int PREC>
__device__ __forceinline__ void disc_levels(double Ac, double Bc, double As, double Bs,
                                            double At, double Bt, double T, int32_t h,
                                            int32_t q, const FieldArgs& f, bool full,
                                            double& w1, double& w2, double& w4) {
  const double cp = PREC == 2 ? f.cphi : f.cphi32;
  const double pc = cp * Ac, ps = cp * As, pt = cp * At;
  double sc = 0.0, ss = 0.0, st = 0.0;
  if constexpr (SPIN) {
    sc = f.cspin * (T / h) * Bc;
    ss = f.cspin * (T / q) * Bs;
    st = f.cspin * (T / q) * Bt;
  }
  w2 = wval<SPIN, PREC>(pc, sc);
  if (full) {
    w4 = 0.5 * (wval<SPIN, PREC>(ps, ss) + wval<SPIN, PREC>(pt, st));
  } else {
    w1 = wval<SPIN, PREC>(0.5 * pc + 0.25 * ps + 0.25 * pt, 0.5 * sc + 0.25 * ss + 0.25 * st);
    w4 = wval<SPIN, PREC>(0.5 * (ps + pt), 0.5 * (ss + st));
  }
}

__device__ __forceinline__ int64_t remap_wg(int32_t w, int32_t n_wg, int32_t n_xcd) {
  // Workgroups are dealt round-robin to the XCDs; give each XCD a
  // contiguous range of logical workgroups so that the items sharing a
  // loop group (same loops, other grid chunks) run under one L2.
  if (n_xcd <= 1) return w;
  const int32_t per = n_wg / n_xcd, rem = n_wg % n_xcd;
  const int32_t xcd = w % n_xcd, idx = w / n_xcd;
  return xcd < rem ? (int64_t)xcd * (per + 1) + idx
                   : (int64_t)rem * (per + 1) + (int64_t)(xcd - rem) * per + idx;
}

// Grid point of lane index p (0 <= p < n_pts): bands of 8 rho rows,
// enumerated T-major inside a band, so that the 64 lanes of a wave cover an
// 8 x 8 tile of (rho, T) (for n_T a multiple of 8) rather than one rho row
// across every T.  The loops of a tile have similar size and offset, so
// fewer waves mix lanes whose segments pass near the axis with lanes whose
// segments stay away from it (each lane's arithmetic is the same either
// way).  A bijection of [0, n_pts).
__device__ __forceinline__ int32_t tile_point(int32_t p, int32_t n_T, int32_t n_pts) {
  constexpr int32_t kB = 8;
  const int32_t n_rho = n_pts / n_T;
  const int32_t band_sz = kB * n_T;
  const int32_t full = n_rho / kB;
  int32_t j, k;
  if (p < full * band_sz) {
    const int32_t band = p / band_sz, q = p - band * band_sz;
    k = q / kB;
    j = band * kB + (q - k * kB);
  } else {
    const int32_t rem = n_rho - full * kB;  // > 0: p < n_pts
    const int32_t q = p - full * band_sz;
    k = q / rem;
    j = full * kB + (q - k * rem);
  }
  return j * n_T + k;
}

// One loop at this lane's grid point: its w is added to acc, and its
// contributions to the scale and rounding accumulators of the mean to a, v
// (loop_scale).  nrm: the loop's norms sqrt(sum c^2), sqrt(sum d_y^2).
template <int KIND, bool SPIN, int PREC>
__device__ __forceinline__ void avg_loop(const float4* __restrict__ seg,
                                         const double4* __restrict__ seg64, float2 nrm,
                                         int32_t n_ppl, int64_t l, double rho, double s,
                                         double T, const LaneF32& c, const FieldArgs& f,
                                         double& acc, double& a, double& v) {
  double A, B, Q, phi, S, cw, ch, R, U;
  if constexpr (PREC == 2) {
    loop_sums_f64<KIND, SPIN, true>(SegArray64{seg64 + l * n_ppl}, n_ppl, rho, s, f, A, B,
                                    Q);
    R = s * s;
    U = rho * s;
  } else {
    if constexpr (PREC == 3)
      loop_sums_f32k<KIND, SPIN>(seg + l * n_ppl, n_ppl, c, f, A, B, Q);
    else
      loop_sums_f32<KIND, SPIN, PREC == 0, 1>(seg + l * n_ppl, n_ppl, c, f, A, B, Q);
    R = KIND == kSech2 ? c.R_s : c.R;
    U = KIND == kSech2 ? c.U_s : c.U;
  }
  epilogue_parts<SPIN, PREC>(A, B, T, n_ppl, f, phi, S, cw, ch);
  const double w = wprod<SPIN>(cw, ch);
  acc += w;
  loop_scale(w, S, cw, ch, phase_l2(Q, n_ppl, R, U, nrm, PREC == 2 ? f.cphi : f.cphi32), a,
             v);
}

// The domain of a grid point: rho_cm >= 0 and T > 0, both finite.
__device__ __forceinline__ bool grid_ok(double rho, double T) {
  return rho >= 0.0 && T > 0.0 && rho < INFINITY && T < INFINITY;
}

// Item decomposition shared by the evaluation kernels: item = (group g,
// loop sub-range, chunk of 64 grid points); loops [l0, l1); the partial
// sums of the item land in row gs = g * n_sub + sub.  Items are numbered
// chunk-minor: consecutive items share their loops.
struct ItemRange {
  int32_t chunk;
  int64_t gs, l0, l1;
};
__device__ __forceinline__ ItemRange item_range(int64_t item, int32_t n_chunks,
                                                int32_t n_sub, int64_t loops_per_group,
                                                int64_t loops_per_sub) {
  ItemRange r;
  r.chunk = (int32_t)(item % n_chunks);
  r.gs = item / n_chunks;
  const int64_t g = r.gs / n_sub;
  const int64_t sub = r.gs % n_sub;
  r.l0 = g * loops_per_group + sub * loops_per_sub;
  r.l1 = r.l0 + loops_per_sub;
  const int64_t gend = (g + 1) * loops_per_group;
  if (r.l1 > gend) r.l1 = gend;
  return r;
}

// One work item of a batch request.  Lane j owns grid point chunk*64 + j and
// accumulates its w over the sub-range's loops in order; the sums land in
// row gs of q.out, q.out_a and q.out_v.
template <int KIND, bool SPIN, int PREC>
__device__ __forceinline__ void run_item(const float4* __restrict__ seg,
                                         const double4* __restrict__ seg64,
                                         const float2* __restrict__ norm, int32_t n_ppl,
                                         const ReqDesc& q, int64_t loops_per_group,
                                         int64_t item) {
  const int32_t lane = threadIdx.x % kWave;
  const ItemRange r = item_range(item, q.n_chunks, q.n_sub, loops_per_group,
                                 q.loops_per_sub);
  const int32_t n_pts = q.n_pts, n_T = q.n_T;
  const int32_t p = r.chunk * kWave + lane;
  const bool valid = p < n_pts;
  const int32_t pg = tile_point(valid ? p : n_pts - 1, n_T, n_pts);
  const double rho = q.rho[pg / n_T];
  const double T = q.T[pg % n_T];
  const double s = sqrt(T);
  const LaneF32 c = lane_consts(rho, s, T, q.f);

  double acc = 0.0, a = 0.0, v = 0.0;
  for (int64_t l = r.l0; l < r.l1; ++l)
    avg_loop<KIND, SPIN, PREC>(seg, seg64, norm[l], n_ppl, l, rho, s, T, c, q.f, acc, a, v);
  if (valid) {
    const int64_t o = r.gs * n_pts + pg;
    q.out[o] = acc;
    q.out_a[o] = a;
    q.out_v[o] = v;
  }
}

// A value every lane of the wave holds, moved to scalar registers, so that
// branches on it are taken by the whole wave.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

constexpr double kEscalate = 0.5e-6;
constexpr double kDecideK = 16.0;

// A flagged point recomputes in FP64 only the sub-range rows whose rounding
// accumulator exceeds thr = B / rows, B being the largest accumulator sum
// that still passes the decision (kDecideK u32 sqrt(B) / N_l = kEscalate
// M_S): the rows left in FP32 then sum to at most rows thr = B, so the
// point's FP32 remainder passes the same test as a point never flagged.
// Where a few loops carry the estimate (a loop through the tube's core
// with a large spin factor) that is a few rows; where every row carries its
// share, all of them.
__device__ __forceinline__ double esc_row_threshold(double ms, int64_t n_loops, int64_t rows) {
  const double b = kEscalate * ms * (double)n_loops / (kDecideK * kU32);
  return b * b / (double)rows;
}

// The FP64 recomputation of the flagged grid points, in work items (row gs
// = g n_sub + sub of the evaluation's partial sums, chunk c of the flagged
// points): the sub-range's loops are walked in FP64 from the raw points
// (loop_sums_f64raw, the FP64 path's arithmetic) for the flagged points
// list[C c .. C c + C - 1] (ascending, cnt of them), and each point's sum
// of w over the sub-range is written over the item's FP32 partial sum.  The
// chunk size C is 64, halved down to 8 while the items would not fill two
// rounds of the chip's wave slots (a few flagged points then still spread
// over every SIMD).  A chunk of more than 32 points takes one per lane, the
// wave walking each loop together (its points come in through scalar loads
// that the wave shares).  A chunk of at most P = 32, 16 or 8 points leaves
// lanes free: the wave's lanes then form R = 64/P copies of the chunk, copy
// r walking loops l0 + r, l0 + r + R, ... through vector loads (R loops per
// wave, so a load touches at most 8 cache lines), and a fixed butterfly
// adds the copies' sums.  Items are numbered chunk-major, k = c rows + gs
// (rows = G n_sub), so that the items of a small count lie side by side and
// spread over every XCD and compute unit.  The split depends only on the
// count, so a request gives the same bits alone and in a batch.
constexpr int kEscWaves = 6;  // waves per SIMD of the recomputation kernels
// two rounds of wave slots: 1024 SIMDs (256 CUs) x kEscWaves, twice
constexpr int64_t kEscFill = 2 * 1024 * kEscWaves;
__device__ __forceinline__ int32_t esc_chunk(int64_t rows, int32_t cnt) {
  int32_t C = kWave;
  while (C > 8 && rows * (((int64_t)cnt + C - 1) / C) < kEscFill) C >>= 1;
  return C;
}
__device__ __forceinline__ int64_t esc_items(int64_t rows, int32_t cnt) {
  const int32_t C = esc_chunk(rows, cnt);
  return rows * (((int64_t)cnt + C - 1) / C);
}

template <int KIND, bool SPIN>
__device__ __forceinline__ void escalate_item(const float* __restrict__ X,
                                              const float* __restrict__ Y, int32_t n_ppl,
                                              const double* __restrict__ rho_g,
                                              const double* __restrict__ T_g, int32_t n_T,
                                              int32_t n_pts, const FieldArgs& f, int64_t k,
                                              int64_t rows, int32_t n_sub,
                                              int64_t loops_per_group, int64_t loops_per_sub,
                                              const int32_t* __restrict__ list, int32_t cnt,
                                              const double* __restrict__ pv,
                                              const double* __restrict__ scale,
                                              double* __restrict__ out) {
  const int32_t chunk = (int32_t)(k / rows);
  const int64_t gs = k % rows;
  const int64_t g = gs / n_sub;
  const int64_t l0 = g * loops_per_group + (gs % n_sub) * loops_per_sub;
  int64_t l1 = l0 + loops_per_sub;
  if (l1 > (g + 1) * loops_per_group) l1 = (g + 1) * loops_per_group;
  const int32_t lane = (int32_t)(threadIdx.x % kWave);
  const int32_t C = esc_chunk(rows, cnt);                // wave-uniform
  const int32_t cnt_c = min(C, cnt - chunk * C);         // 1 .. C
  const int32_t P = cnt_c <= 8 ? 8 : cnt_c <= 16 ? 16 : cnt_c <= 32 ? 32 : kWave;
  const int32_t p = lane % P, r = lane / P;
  const bool esc = p < cnt_c;
  const int32_t pg = list[chunk * C + (esc ? p : cnt_c - 1)];
  // only the rows that carry the point's estimate are recomputed; an item
  // none of whose points needs its row does nothing
  const int64_t n_loops = loops_per_group * (rows / n_sub);
  const bool need = esc && pv[gs * n_pts + pg] > esc_row_threshold(scale[pg], n_loops, rows);
  if (__ballot(need) == 0) return;
  const double rho = rho_g[pg / n_T];
  const double T = T_g[pg % n_T];
  const double s = sqrt(T);
  double acc = 0.0;
  if (P == kWave) {
    for (int64_t l = l0; l < l1; ++l) {
      double A, B, phi, S;
      // (wave_uniform keeps the compiler from merging this walk with the
      // copies' below, which would make these loads vector loads)
      const int64_t lu = wave_uniform(l);
      loop_sums_f64raw<KIND, SPIN>(X + lu * n_ppl, Y + lu * n_ppl, n_ppl, 0, 1, n_ppl, rho,
                                   s, f, A, B);
      acc += epilogue<SPIN, 2>(A, B, T, n_ppl, f, phi, S);
    }
  } else {
    const int32_t R = kWave / P;
    for (int64_t l = l0 + r; l < l1; l += R) {
      double A, B, phi, S;
      loop_sums_f64raw<KIND, SPIN>(X + l * n_ppl, Y + l * n_ppl, n_ppl, 0, 1, n_ppl, rho, s,
                                   f, A, B);
      acc += epilogue<SPIN, 2>(A, B, T, n_ppl, f, phi, S);
    }
    if (P == 8) acc += __shfl_xor(acc, 8);
    if (P <= 16) acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
  }
  if (need && r == 0) out[gs * n_pts + pg] = acc;
}

// The flagged grid points of one evaluation in ascending order, list[0 ..
// count), by one workgroup of kCompactThreads: per tile of that many points
// a wave ballot and popcount give each flagged point its rank.  Four waves:
// a workgroup this small finds room on a compute unit beside another
// server slot's persistent batch kernel as soon as one wave per SIMD drains.
constexpr int kCompactThreads = 256;
__device__ __forceinline__ void compact_flags(const uint8_t* __restrict__ flags,
                                              int32_t n_pts, int32_t* __restrict__ list,
                                              int32_t* __restrict__ count) {
  constexpr int kWaves = kCompactThreads / kWave;
  __shared__ int32_t wave_cnt[kWaves];
  const int32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  int32_t base = 0;
  for (int32_t t0 = 0; t0 < n_pts; t0 += kCompactThreads) {
    const int32_t p = t0 + (int32_t)threadIdx.x;
    const bool fl = p < n_pts && flags[p] != 0;
    const uint64_t m = __ballot(fl);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int32_t off = base, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (w < wave) off += wave_cnt[w];
      tot += wave_cnt[w];
    }
    if (fl) list[off + __popcll(m & ((1ull << lane) - 1))] = p;
    __syncthreads();  // wave_cnt is rewritten by the next tile
    base += tot;
  }
  if (threadIdx.x == 0) *count = base;
}

// Per grid point p of one evaluation, from the partial sums pa, pv
// ([rows][n_pts], rows = G n_sub) of loop_scale's accumulators:
//   ms  the scale M_S = (1/N_l) sum_l |w_l| max(1, S_l),
//   fe  the stated rounding-error estimate of the mean,
//       kPhaseK u sqrt(sum_l v_l) / N_l + kSysK u M_S (u of the precision),
//   esc whether the point is recomputed in FP64 (compensated FP32 only):
//       when kDecideK u sqrt(sum_l v_l) / N_l exceeds kEscalate M_S, half
//       the mean tolerance 1e-6 M_S; the estimate then takes FP64's u.
// kDecideK is the decision's calibration: the largest mean error measured
// against the FP64 oracle on the stress fields (1024 loops of 8192 points,
// every sech^2 tube) is 3.1 u sqrt(sum_l v_l) / N_l, and a single loop's
// phase error stays below 18 u sqrt(sum_i t_i^2); at kDecideK = 16 a point
// left in FP32 is then within half the tolerance even when one loop
// carries the mean.
__device__ __forceinline__ void scale_point(const double* __restrict__ pa,
                                            const double* __restrict__ pv, int64_t rows,
                                            int32_t n_pts, int64_t n_loops, int32_t prec,
                                            int32_t p, double& ms, double& fe, bool& esc) {
  double sa = 0.0, sv = 0.0;
  for (int64_t r = 0; r < rows; ++r) {
    sa += pa[r * n_pts + p];
    sv += pv[r * n_pts + p];
  }
  ms = sa / (double)n_loops;
  const double u = prec == 2 ? kU64 : kU32;
  const double rnd = u * sqrt(sv) / (double)n_loops;
  esc = prec == 0 && kDecideK * rnd > kEscalate * ms;
  if (!esc) {
    fe = kPhaseK * rnd + kSysK * u * ms;
  } else {
    // the rows left in FP32 (esc_row_threshold) and their estimate
    const double thr = esc_row_threshold(ms, n_loops, rows);
    double rest = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
      const double v = pv[r * n_pts + p];
      if (!(v > thr)) rest += v;
    }
    fe = kPhaseK * u * sqrt(rest) / (double)n_loops + kSysK * u * ms;
  }
}

// ------------------------------------------------------------- kernels
// One workgroup = avg_waves(PREC) consecutive items, normally chunks of one
// (group, sub-range): they walk the same loops, and a barrier after every
// loop keeps them in step so that a loop's segments are fetched from HBM
// about once per workgroup and then served from the caches.  Every wave,
// including padding waves past the last item, runs the same
// loops_per_sub barrier iterations.
// Register budget 64 VGPRs, 8 waves per SIMD: the FP32 kernels (77
// uncapped, 6 waves) then spill three per-item values, reloaded after the
// item's last loop; the FP64 ones need at most 60 (their polynomial
// coefficients are scalar operands), 8 waves in workgroups of 4.
template <int KIND, bool SPIN, int PREC>
__global__ __launch_bounds__(avg_waves(PREC) * kWave)
__attribute__((amdgpu_waves_per_eu(8))) void k_average(
    const float4* __restrict__ seg, const double4* __restrict__ seg64,
    const float2* __restrict__ norm, int32_t n_ppl,
    const double* __restrict__ rho_g, const double* __restrict__ T_g,
    int32_t n_T, int32_t n_pts, FieldArgs f, Sched sc,
    double* __restrict__ out, double* __restrict__ out_a, double* __restrict__ out_v) {
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t lane = threadIdx.x % kWave;
  const int64_t item = remap_wg(blockIdx.x, sc.n_wg, sc.n_xcd) * avg_waves(PREC) + wave;
  const bool live = item < sc.n_items;
  ItemRange r = item_range(live ? item : 0, sc.n_chunks, sc.n_sub, sc.loops_per_group,
                           sc.loops_per_sub);
  if (!live) r.l1 = r.l0;

  const int32_t p = r.chunk * kWave + lane;
  const bool valid = live && p < n_pts;
  const int32_t pg = tile_point(p < n_pts ? p : n_pts - 1, n_T, n_pts);
  const double rho = rho_g[pg / n_T];
  const double T = T_g[pg % n_T];
  const double s = sqrt(T);
  const LaneF32 c = lane_consts(rho, s, T, f);

  double acc = 0.0, a = 0.0, v = 0.0;
  for (int64_t k = 0; k < sc.loops_per_sub; ++k) {
    const int64_t l = r.l0 + k;
    if (l < r.l1)
      avg_loop<KIND, SPIN, PREC>(seg, seg64, norm[l], n_ppl, l, rho, s, T, c, f, acc, a, v);
    __syncthreads();
  }
  if (valid) {
    const int64_t o = r.gs * n_pts + pg;
    // a grid point outside the domain (device grids are not validated on
    // the host) gives NaN, whatever its arithmetic produced
    const double bad = grid_ok(rho, T) ? 0.0 : NAN;
    out[o] = acc + bad;
    out_a[o] = a + bad;
    out_v[o] = v + bad;
  }
}

// FP64 recomputation of the flagged grid points of an evaluation: the
// esc_items(G n_sub, count) items of escalate_item, grid-stride (four waves
// per workgroup, no barrier).  Register budget 84 VGPRs, 6 waves per SIMD
// (the sech^2 spinor walk needs 80).
template <int KIND, bool SPIN>
__global__ __launch_bounds__(kWavesPerWG * kWave)
__attribute__((amdgpu_waves_per_eu(kEscWaves))) void k_escalate(
    const float* __restrict__ X, const float* __restrict__ Y, int32_t n_ppl,
    const double* __restrict__ rho_g, const double* __restrict__ T_g, int32_t n_T,
    int32_t n_pts, FieldArgs f, Sched sc, const int32_t* __restrict__ list,
    const int32_t* __restrict__ count, const double* __restrict__ pv,
    const double* __restrict__ scale, double* __restrict__ out) {
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t cnt = __builtin_amdgcn_readfirstlane(*count);
  const int64_t rows = sc.n_items / sc.n_chunks;
  const int64_t total = esc_items(rows, cnt);
  for (int64_t k = (int64_t)blockIdx.x * kWavesPerWG + wave; k < total;
       k += (int64_t)gridDim.x * kWavesPerWG)
    escalate_item<KIND, SPIN>(X, Y, n_ppl, rho_g, T_g, n_T, n_pts, f, k, rows, sc.n_sub,
                              sc.loops_per_group, sc.loops_per_sub, list, cnt, pv, scale,
                              out);
}

// The flagged points of one evaluation, compacted (compact_flags).
__global__ __launch_bounds__(kCompactThreads) void k_compact(const uint8_t* __restrict__ flags,
                                                             int32_t n_pts,
                                                             int32_t* __restrict__ list,
                                                             int32_t* __restrict__ count) {
  compact_flags(flags, n_pts, list, count);
}

// Scale, rounding estimate and escalation flag per grid point of one
// evaluation (scale_point); scale and fp_err may be NULL.
__global__ __launch_bounds__(256) void k_scale(const double* __restrict__ pa,
                                               const double* __restrict__ pv, int64_t rows,
                                               int32_t n_pts, int64_t n_loops, int32_t prec,
                                               double* __restrict__ scale,
                                               double* __restrict__ fp_err,
                                               uint8_t* __restrict__ flags) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  double ms, fe;
  bool esc;
  scale_point(pa, pv, rows, n_pts, n_loops, prec, p, ms, fe, esc);
  if (scale) scale[p] = ms;
  if (fp_err) fp_err[p] = fe;
  flags[p] = esc ? 1 : 0;
}

// Discretisation estimate (Sec. 4.1): the schedule, workgroup shape and
// barrier of k_average, with the loop split into its circle, square and
// triangle sub-loops (from the sub-loop segment array, `sub` for the FP32
// paths, `sub64` for FP64) and three accumulators, one per level (N, N/2,
// N/4).  With `full`, the N level is the whole loop (segment array `seg` or
// `seg64`), which doubles the segment work.  Output level k of item gs lands
// in out[(k * G * n_sub + gs) * n_pts + p].
// The FP32 kernels are held to 80 VGPRs (6 waves per SIMD, three 8-wave
// workgroups per CU): their three sets of sums need ~100, which would leave
// room for two workgroups, and the few values spilled to scratch (live
// across the sub-loop walks, not inside them) cost less than the lost
// occupancy.  The FP64 kernels need at most 75 and run at the same 6
// waves per SIMD, spilling nothing inside a segment walk.
template <int KIND, bool SPIN, int PREC>
__global__ __launch_bounds__(avg_waves(PREC) * kWave)
__attribute__((amdgpu_waves_per_eu(6))) void k_disc(
    const float4* __restrict__ seg, const float4* __restrict__ sub,
    const double4* __restrict__ seg64, const double4* __restrict__ sub64, int32_t n_ppl,
    const double* __restrict__ rho_g, const double* __restrict__ T_g,
    int32_t n_T, int32_t n_pts, FieldArgs f, Sched sc, int32_t full,
    double* __restrict__ out) {
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t lane = threadIdx.x % kWave;
  const int64_t item = remap_wg(blockIdx.x, sc.n_wg, sc.n_xcd) * avg_waves(PREC) + wave;
  const bool live = item < sc.n_items;
  const int64_t it = live ? item : 0;
  const int32_t chunk = (int32_t)(it % sc.n_chunks);
  const int64_t gs = it / sc.n_chunks;  // g * n_sub + sub
  const int64_t g = gs / sc.n_sub;
  const int64_t sr = gs % sc.n_sub;
  const int64_t l0 = g * sc.loops_per_group + sr * sc.loops_per_sub;
  int64_t l1 = l0 + sc.loops_per_sub;
  const int64_t gend = (g + 1) * sc.loops_per_group;
  if (l1 > gend) l1 = gend;
  if (!live) l1 = l0;

  const int32_t p = chunk * kWave + lane;
  const bool valid = live && p < n_pts;
  const int32_t pg = tile_point(p < n_pts ? p : n_pts - 1, n_T, n_pts);
  const double rho = rho_g[pg / n_T];
  const double T = T_g[pg % n_T];
  const double s = sqrt(T);
  const LaneF32 c = lane_consts(rho, s, T, f);
  const int32_t h = n_ppl / 2, q = n_ppl / 4;

  double acc1 = 0.0, acc2 = 0.0, acc4 = 0.0;
  for (int64_t k = 0; k < sc.loops_per_sub; ++k) {
    const int64_t l = l0 + k;
    if (l < l1) {
      double Ac, Bc, As, Bs, At, Bt;
      if constexpr (PREC == 2) {
        const double4* u = sub64 + l * n_ppl;
        loop_sums_f64seg<KIND, SPIN>(u, h, rho, s, f, Ac, Bc);
        loop_sums_f64seg<KIND, SPIN>(u + h, q, rho, s, f, As, Bs);
        loop_sums_f64seg<KIND, SPIN>(u + h + q, q, rho, s, f, At, Bt);
      } else {
        const float4* u = sub + l * n_ppl;
        double Q;
        loop_sums_f32<KIND, SPIN, PREC == 0>(u, h, c, f, Ac, Bc, Q);
        loop_sums_f32<KIND, SPIN, PREC == 0>(u + h, q, c, f, As, Bs, Q);
        loop_sums_f32<KIND, SPIN, PREC == 0>(u + h + q, q, c, f, At, Bt, Q);
      }
      double w1 = 0.0, w2, w4;
      disc_levels<SPIN, PREC>(Ac, Bc, As, Bs, At, Bt, T, h, q, f, full != 0, w1, w2, w4);
      if (full) {
        double A, B, phi, S;
        if constexpr (PREC == 2) {
          loop_sums_f64seg<KIND, SPIN>(seg64 + l * n_ppl, n_ppl, rho, s, f, A, B);
        } else {
          double Q;
          loop_sums_f32<KIND, SPIN, PREC == 0>(seg + l * n_ppl, n_ppl, c, f, A, B, Q);
        }
        w1 = epilogue<SPIN, PREC>(A, B, T, n_ppl, f, phi, S);
      }
      acc1 += w1;
      acc2 += w2;
      acc4 += w4;
    }
    __syncthreads();
  }
  if (valid) {
    const int64_t L = sc.n_items / sc.n_chunks;  // G * n_sub
    out[gs * n_pts + pg] = acc1;
    out[(L + gs) * n_pts + pg] = acc2;
    out[(2 * L + gs) * n_pts + pg] = acc4;
  }
}

// Next item of a persistent wavefront's work loop: one increment of the
// counter per wave, whose old value every lane receives.  Every lane
// executes the atomic (lane 0 adds 1, the others 0; the compiler folds the
// wave's lanes into one memory operation), so that no lane-dependent branch
// sits in the loop: around a branch on the lane the compiler may send lanes
// 1..63 from the end of one item straight back to the broadcast, where they
// then run without lane 0 and read a stale item.
__device__ __forceinline__ int64_t take_item(unsigned int* counter) {
  const unsigned int t = atomicAdd(counter, threadIdx.x % kWave == 0 ? 1u : 0u);
  return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)t);
}

// Batched evaluation of uneven requests in one persistent launch.  Items of
// all requests form one index space (request r owns [item_begin_r,
// item_begin_r + n_items_r)); each wavefront repeatedly takes the next item
// from a device counter until the counter passes the total, so every wave
// exits once the work is handed out.  An item's output slot is fixed by its
// index, so results do not depend on which wave ran it.
// The FP32 batch kernel is held to 64 VGPRs (8 waves per SIMD instead of
// 5 at its 86): more waves hide the scalar-load and dispatch latencies of
// the persistent item loop better than the spills it costs (measured
// 2.20e12 -> 2.50e12 segment-evals/s on a 128-request batch).  The FP64
// one runs at the same 8 waves (it needs 64 VGPRs, two per-item values
// spilled outside the walks).
template <int PREC>
__global__ __launch_bounds__(kWavesPerWG * kWave)
__attribute__((amdgpu_waves_per_eu(8))) void k_batch(
    const float4* __restrict__ seg, const double4* __restrict__ seg64,
    const float2* __restrict__ norm, int32_t n_ppl, const BatchHeader* __restrict__ hdr,
    unsigned int* __restrict__ counter, int64_t loops_per_group) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  const int64_t total_items = hdr->total_items;
  for (;;) {
    const int64_t item = take_item(counter);
    if (item >= total_items) break;
    // request owning the item: last r with item_begin <= item
    int32_t lo = 0, hi = n_reqs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (reqs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    const ReqDesc& q = reqs[lo];
    const int64_t li = item - q.item_begin;
    switch (q.f.kind * 2 + q.spin) {
#define WL_ITEM(K, SP) run_item<K, SP, PREC>(seg, seg64, norm, n_ppl, q, loops_per_group, li)
      case 0: WL_ITEM(kConst, false); break;
      case 1: WL_ITEM(kConst, true); break;
      case 2: WL_ITEM(kSech2, false); break;
      case 3: WL_ITEM(kSech2, true); break;
      case 4: WL_ITEM(kGauss, false); break;
      case 5: WL_ITEM(kGauss, true); break;
      case 6: WL_ITEM(kRational, false); break;
      default: WL_ITEM(kRational, true); break;
#undef WL_ITEM
    }
  }
}

// FP64 recomputation of the flagged grid points of a compensated-FP32
// batch, one kernel per field kind and spin (a kernel holding every
// variant would spill inside the segment walks): a persistent loop over the
// escalate_item items of the batch's requests of that variant, taken from
// the variant's work counter; the header's esc_begin table of the variant,
// [n_reqs + 1], holds the first item of each request (k_esc_begin; requests
// of other variants have none).
constexpr int kVariants = 8;  // field kind x spin
template <int KIND, bool SPIN>
__global__ __launch_bounds__(kWavesPerWG * kWave)
__attribute__((amdgpu_waves_per_eu(kEscWaves))) void k_escalate_batch(
    const float* __restrict__ X, const float* __restrict__ Y, int32_t n_ppl,
    const BatchHeader* __restrict__ hdr, unsigned int* __restrict__ counter,
    int32_t n_groups, int64_t loops_per_group) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  const int64_t* __restrict__ esc_begin =
      hdr->esc_begin + (int64_t)(KIND * 2 + (SPIN ? 1 : 0)) * (n_reqs + 1);
  // the table is written by an earlier kernel, so its entries come in
  // through vector loads: wave_uniform keeps the loop's branches scalar
  const int64_t total = wave_uniform(esc_begin[n_reqs]);
  for (;;) {
    const int64_t item = take_item(counter);
    if (item >= total) break;
    // request owning the item: last r with esc_begin[r] <= item (a request
    // without items has the same entry as the next one and is passed over)
    int32_t lo = 0, hi = n_reqs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (wave_uniform(esc_begin[mid]) <= item) lo = mid; else hi = mid - 1;
    }
    const ReqDesc& q = reqs[lo];
    const int32_t cnt = __builtin_amdgcn_readfirstlane(*q.count);
    escalate_item<KIND, SPIN>(X, Y, n_ppl, q.rho, q.T, q.n_T, q.n_pts, q.f,
                              item - wave_uniform(esc_begin[lo]), (int64_t)n_groups * q.n_sub,
                              q.n_sub, loops_per_group, q.loops_per_sub, q.list, cnt, q.out_v,
                              q.scale, q.out);
  }
}

// First recomputation item of each request of a batch, per variant (one
// thread, in request order): for the request's variant v,
// esc_begin[v][r + 1] = esc_begin[v][r] + esc_items(G n_sub_r, count_r);
// the other variants' tables repeat their entry.
__global__ void k_esc_begin(const BatchHeader* __restrict__ hdr, int32_t n_groups,
                            int64_t loops_per_group) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  int64_t* __restrict__ esc_begin = hdr->esc_begin;
  int64_t acc[kVariants];
  for (int v = 0; v < kVariants; ++v) {
    acc[v] = 0;
    esc_begin[(int64_t)v * (n_reqs + 1)] = 0;
  }
  for (int32_t r = 0; r < n_reqs; ++r) {
    const int v = reqs[r].f.kind * 2 + (reqs[r].spin ? 1 : 0);
    acc[v] += esc_items((int64_t)n_groups * reqs[r].n_sub, *reqs[r].count);
    for (int u = 0; u < kVariants; ++u) esc_begin[(int64_t)u * (n_reqs + 1) + r + 1] = acc[u];
  }
}

// The flagged points of every request of a batch, compacted: one workgroup
// per request (grid-stride over the requests).
__global__ __launch_bounds__(kCompactThreads) void k_compact_batch(
    const BatchHeader* __restrict__ hdr) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  for (int32_t r = blockIdx.x; r < n_reqs; r += gridDim.x) {
    const ReqDesc& q = reqs[r];
    compact_flags(q.flags, q.n_pts, q.list, q.count);
    __syncthreads();
  }
}

// Scale, rounding estimate and escalation flag of every grid point of a
// batch (thread t handles point t of the concatenation over requests).
__global__ __launch_bounds__(256) void k_scale_batch(const BatchHeader* __restrict__ hdr,
                                                     int32_t n_groups, int64_t n_loops,
                                                     int32_t prec) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  const int64_t total_pts = hdr->total_pts;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total_pts;
       t += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n_reqs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (reqs[mid].pts_begin <= t) lo = mid; else hi = mid - 1;
    }
    const ReqDesc& q = reqs[lo];
    const int32_t p = (int32_t)(t - q.pts_begin);
    double ms, fe;
    bool esc;
    scale_point(q.out_a, q.out_v, (int64_t)n_groups * q.n_sub, q.n_pts, n_loops, prec, p,
                ms, fe, esc);
    q.scale[p] = ms;
    q.fp_err[p] = fe;
    q.flags[p] = esc ? 1 : 0;
  }
}

// Batched sub-range reduction and statistics: thread t handles output t of
// the concatenation over requests (binary search for its request).
// Result region of a batch: [group sums | means | errors | partials].
__global__ __launch_bounds__(256) void k_reduce_batch(const BatchHeader* __restrict__ hdr,
                                                      double* __restrict__ sums) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  const int64_t total = hdr->total_sums;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n_reqs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (reqs[mid].sums_begin <= t) lo = mid; else hi = mid - 1;
    }
    const ReqDesc& q = reqs[lo];
    if (q.n_sub == 1) continue;  // written directly by the item kernel
    const int64_t o = t - q.sums_begin;
    const int64_t g = o / q.n_pts, p = o % q.n_pts;
    double acc = 0.0;
    for (int32_t s = 0; s < q.n_sub; ++s) acc += q.out[(g * q.n_sub + s) * q.n_pts + p];
    sums[t] = acc;
  }
}

__device__ __forceinline__ void stats_point(const double* __restrict__ sums,
                                            int32_t n_groups, int32_t n_pts,
                                            int64_t n_loops, int32_t p, double& m,
                                            double& e) {
  double tot = 0.0;
  for (int32_t g = 0; g < n_groups; ++g) tot += sums[(int64_t)g * n_pts + p];
  m = tot / (double)n_loops;
  const double per = (double)(n_loops / n_groups);
  double ss = 0.0;
  for (int32_t g = 0; g < n_groups; ++g) {
    const double d = sums[(int64_t)g * n_pts + p] / per - m;
    ss += d * d;
  }
  e = n_groups > 1 ? sqrt(ss / ((double)n_groups * (n_groups - 1))) : NAN;
}

__global__ __launch_bounds__(256) void k_stats_batch(const BatchHeader* __restrict__ hdr,
                                                     int32_t n_groups, int64_t n_loops,
                                                     double* __restrict__ res) {
  const ReqDesc* __restrict__ reqs =
      (const ReqDesc*)((const char*)hdr + kBatchDescOffset);
  const int32_t n_reqs = (int32_t)hdr->n_reqs;
  const int64_t total_pts = hdr->total_pts;
  const double* __restrict__ sums = res;
  double* __restrict__ mean = res + hdr->total_sums;
  double* __restrict__ err = mean + total_pts;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total_pts;
       t += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n_reqs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (reqs[mid].pts_begin <= t) lo = mid; else hi = mid - 1;
    }
    const ReqDesc& q = reqs[lo];
    double m, e;
    stats_point(sums + q.sums_begin, n_groups, q.n_pts, n_loops,
                (int32_t)(t - q.pts_begin), m, e);
    mean[t] = m;
    err[t] = e;
  }
}

// Clears the work counters of a batch (one thread per counter): a kernel,
// not a memset node, so that captured graphs replay it reliably.
__global__ void k_zero_u32(unsigned int* __restrict__ p) { p[threadIdx.x] = 0u; }

// Per-loop values of the (sub-)loop that takes, within each loop of the
// ensemble, segments seg_off .. seg_off+m-1 of `seg` (FP32 paths) or of
// `seg64` (FP64 path).  Compensated FP32: each lane's phase carries the
// rounding estimate kPhaseK u sqrt(sum_i e_i^2) over its segment terms,
// e_i = (|R c_i| + |U d_y,i|) qe_i the size of term i's rounding relative
// to u: the cross product's parts R c_i and U d_y,i are summed apart (and
// cancel where a loop crosses the axis far from its centre), and qe_i is
// qa_i or, where qa_i is the difference of two larger parts, their size
// (field_f32); where it exceeds the phase tolerance
// 1e-5 max(1, |Phi|)
// the lane's phase, spin exponent and w are recomputed in FP64 from the raw
// points (the whole wave walks the loop when any lane is flagged).
template <int KIND, bool SPIN, int PREC>
__global__ __launch_bounds__(kWavesPerWG * kWave) void k_per_loop(
    const float4* __restrict__ seg, const double4* __restrict__ seg64,
    const float* __restrict__ X, const float* __restrict__ Y, int32_t n_ppl,
    SubLoop sl,
    const double* __restrict__ rho_g, const double* __restrict__ T_g,
    int32_t n_T, int32_t n_pts, int32_t n_chunks, FieldArgs f, int64_t loop0,
    int64_t n_loops, double* __restrict__ o_phase, double* __restrict__ o_spin,
    double* __restrict__ o_w) {
  const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t lane = threadIdx.x % kWave;
  const int64_t item = (int64_t)blockIdx.x * kWavesPerWG + wave;
  if (item >= n_loops * n_chunks) return;
  const int64_t li = item / n_chunks;
  const int32_t chunk = (int32_t)(item % n_chunks);
  const int64_t l = loop0 + li;
  const int32_t p = chunk * kWave + lane;
  const bool valid = p < n_pts;
  const int32_t pp = valid ? p : n_pts - 1;
  const double rho = rho_g[pp / n_T];
  const double T = T_g[pp % n_T];
  const double s = sqrt(T);
  const LaneF32 c = lane_consts(rho, s, T, f);
  double A, B, Q, phi, S;
  if constexpr (PREC == 2) {
    loop_sums_f64seg<KIND, SPIN>(seg64 + l * n_ppl + sl.seg_off, sl.m, rho, s, f, A, B);
  } else if constexpr (PREC == 3) {
    loop_sums_f32k<KIND, SPIN>(seg + l * n_ppl + sl.seg_off, sl.m, c, f, A, B, Q);
  } else {
    loop_sums_f32<KIND, SPIN, PREC == 0, PREC == 0 ? 2 : 0>(seg + l * n_ppl + sl.seg_off,
                                                            sl.m, c, f, A, B, Q);
  }
  double w = epilogue<SPIN, PREC>(A, B, T, sl.m, f, phi, S);
  if constexpr (PREC == 0) {
    const double l2 = fabs(f.cphi32) * sqrt(Q);
    const bool esc = valid && kPhaseK * kU32 * l2 > 1e-5 * fmax(1.0, fabs(phi));
    if (__ballot(esc) != 0) {
      double A64, B64, phi64, S64;
      loop_sums_f64raw<KIND, SPIN>(X + l * n_ppl, Y + l * n_ppl, n_ppl, sl.first, sl.stride,
                                   sl.m, rho, s, f, A64, B64);
      const double w64 = epilogue<SPIN, 2>(A64, B64, T, sl.m, f, phi64, S64);
      if (esc) {
        phi = phi64;
        S = S64;
        w = w64;
      }
    }
  }
  if (valid) {
    const int64_t o = li * n_pts + p;
    o_phase[o] = phi;
    o_spin[o] = S;
    o_w[o] = w;
  }
}

// Loop norms sqrt(sum_i c_i^2), sqrt(sum_i d_y,i^2) of every loop's segment
// array (the rounding estimate's geometry factors): one wavefront per loop,
// lanes striding over its segments, FP64 sums combined across the wave.
__global__ __launch_bounds__(256) void k_norms(const float4* __restrict__ seg,
                                               int64_t n_loops, int32_t n_ppl,
                                               float2* __restrict__ norm) {
  const int32_t lane = threadIdx.x % kWave;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t l = w0; l < n_loops; l += nw) {
    double cc = 0.0, dd = 0.0;
    for (int32_t i = lane; i < n_ppl; i += kWave) {
      const float4 q = seg[l * n_ppl + i];
      cc += (double)q.w * (double)q.w;
      dd += (double)q.z * (double)q.z;
    }
    for (int32_t off = kWave / 2; off > 0; off >>= 1) {
      cc += __shfl_xor(cc, off);
      dd += __shfl_xor(dd, off);
    }
    if (lane == 0) norm[l] = make_float2((float)sqrt(cc), (float)sqrt(dd));
  }
}

// Per-segment unit quantities (see wl_internal.h) of the segment from
// (x0, y0) to (x1, y1), formed in FP64 and rounded once to FP32.
__device__ __forceinline__ float4 seg_quantities(float x0f, float y0f, float x1f, float y1f) {
  const double x0 = x0f, y0 = y0f, x1 = x1f, y1 = y1f;
  float4 o;
  o.x = (float)(0.5 * (x0 + x1));
  o.y = (float)(0.25 * (y0 + y1) * (y0 + y1));
  o.z = (float)(y1 - y0);
  o.w = (float)(x0 * y1 - y0 * x1);
  return o;
}

// Segment array of every loop (segment i: point i -> i+1 mod N); flags
// non-finite input.
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ X,
                                              const float* __restrict__ Y,
                                              int64_t n_loops, int32_t n_ppl,
                                              float4* __restrict__ seg,
                                              int* __restrict__ bad) {
  const int64_t total = n_loops * n_ppl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / n_ppl;
    const int32_t i = (int32_t)(t % n_ppl);
    const int32_t j = (i + 1 == n_ppl) ? 0 : i + 1;
    const float x0f = X[l * n_ppl + i], y0f = Y[l * n_ppl + i];
    const float x1f = X[l * n_ppl + j], y1f = Y[l * n_ppl + j];
    if (!isfinite(x0f) || !isfinite(y0f)) *bad = 1;
    seg[t] = seg_quantities(x0f, y0f, x1f, y1f);
  }
}

// FP64 segment array of every loop (segment i: point i -> i+1 mod N).
__global__ __launch_bounds__(256) void k_prep64(const float* __restrict__ X,
                                                const float* __restrict__ Y,
                                                int64_t n_loops, int32_t n_ppl,
                                                double4* __restrict__ seg) {
  const int64_t total = n_loops * n_ppl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / n_ppl;
    const int32_t i = (int32_t)(t % n_ppl);
    const int32_t j = (i + 1 == n_ppl) ? 0 : i + 1;
    seg[t] = seg_quantities64(X[l * n_ppl + i], Y[l * n_ppl + i], X[l * n_ppl + j],
                              Y[l * n_ppl + j]);
  }
}

// Sub-loop segment layout (N divisible by 4), N entries per loop: [0, N/2)
// the circle sub-loop (point 2j -> 2j+2), [N/2, 3N/4) the square one
// (4j+1 -> 4j+5), [3N/4, N) the triangle one (4j+3 -> 4j+7), point indices
// mod N.  Entry i runs from point a to point b.
__device__ __forceinline__ void sub_endpoints(int32_t i, int32_t n_ppl, int32_t& a,
                                              int32_t& b) {
  const int32_t h = n_ppl / 2, q = n_ppl / 4;
  int32_t step;
  if (i < h) {
    a = 2 * i;
    step = 2;
  } else if (i < h + q) {
    a = 4 * (i - h) + 1;
    step = 4;
  } else {
    a = 4 * (i - h - q) + 3;
    step = 4;
  }
  b = a + step;
  if (b >= n_ppl) b -= n_ppl;
}

// Sub-loop segment array of every loop, FP32 quantities.
__global__ __launch_bounds__(256) void k_prep_sub(const float* __restrict__ X,
                                                  const float* __restrict__ Y,
                                                  int64_t n_loops, int32_t n_ppl,
                                                  float4* __restrict__ sub) {
  const int64_t total = n_loops * n_ppl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / n_ppl;
    int32_t a, b;
    sub_endpoints((int32_t)(t % n_ppl), n_ppl, a, b);
    const float* x = X + l * n_ppl;
    const float* y = Y + l * n_ppl;
    sub[t] = seg_quantities(x[a], y[a], x[b], y[b]);
  }
}

// Sub-loop segment array of every loop, FP64 quantities.
__global__ __launch_bounds__(256) void k_prep_sub64(const float* __restrict__ X,
                                                    const float* __restrict__ Y,
                                                    int64_t n_loops, int32_t n_ppl,
                                                    double4* __restrict__ sub) {
  const int64_t total = n_loops * n_ppl;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = t / n_ppl;
    int32_t a, b;
    sub_endpoints((int32_t)(t % n_ppl), n_ppl, a, b);
    const float* x = X + l * n_ppl;
    const float* y = Y + l * n_ppl;
    sub[t] = seg_quantities64(x[a], y[a], x[b], y[b]);
  }
}

__global__ __launch_bounds__(256) void k_reduce_sub(const double* __restrict__ part,
                                                    int32_t n_groups, int32_t n_sub,
                                                    int32_t n_pts,
                                                    double* __restrict__ sums) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_groups * n_pts) return;
  const int64_t g = t / n_pts, p = t % n_pts;
  double acc = 0.0;
  for (int32_t s = 0; s < n_sub; ++s) acc += part[(g * n_sub + s) * n_pts + p];
  sums[t] = acc;
}

// Mean and standard error of the group means (Sec. 4.2.3) per grid point.
__global__ __launch_bounds__(256) void k_stats(const double* __restrict__ sums,
                                               int32_t n_groups, int32_t n_pts,
                                               int64_t n_loops,
                                               double* __restrict__ mean,
                                               double* __restrict__ err) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  double m, e;
  stats_point(sums, n_groups, n_pts, n_loops, p, m, e);
  if (mean) mean[p] = m;
  if (err) err[p] = e;
}

// Discretisation estimate, per grid point: the extrapolated level's group
// sums (8/3 W_N - 2 W_N/2 + 1/3 W_N/4, group by group, written as level 3),
// then mean and group standard error of the four levels and
// delta = |W_N - W_inf| (Sec. 4.1).  sums: [4][G][n_pts].
__global__ __launch_bounds__(256) void k_disc_finish(double* __restrict__ sums,
                                                     int32_t n_groups, int32_t n_pts,
                                                     int64_t n_loops,
                                                     double* __restrict__ mean,
                                                     double* __restrict__ err,
                                                     double* __restrict__ delta) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  const int64_t L = (int64_t)n_groups * n_pts;
  for (int32_t g = 0; g < n_groups; ++g) {
    const int64_t o = (int64_t)g * n_pts + p;
    sums[3 * L + o] = (8.0 * sums[o] - 6.0 * sums[L + o] + sums[2 * L + o]) / 3.0;
  }
  double m0 = 0.0, m3 = 0.0;
  for (int32_t k = 0; k < 4; ++k) {
    double m, e;
    stats_point(sums + k * L, n_groups, n_pts, n_loops, p, m, e);
    if (mean) mean[(int64_t)k * n_pts + p] = m;
    if (err) err[(int64_t)k * n_pts + p] = e;
    if (k == 0) m0 = m;
    if (k == 3) m3 = m;
  }
  if (delta) delta[p] = fabs(m0 - m3);
}

// ------------------------------------------------------------ dispatch
template <int KIND, bool SPIN, int PREC>
hipError_t launch_avg_t(const FieldArgs& f, const float4* seg, const double4* seg64,
                        const float2* norm, int32_t n_ppl, const double* rho,
                        const double* T, int32_t n_T, int32_t n_pts, const Sched& s0,
                        double* out, double* out_a, double* out_v, hipStream_t st) {
  if ((PREC == 2 ? seg64 == nullptr : seg == nullptr) || norm == nullptr)
    return hipErrorInvalidValue;
  Sched s = s0;
  s.n_wg = (int32_t)((s.n_items + avg_waves(PREC) - 1) / avg_waves(PREC));
  hipLaunchKernelGGL((k_average<KIND, SPIN, PREC>), dim3(s.n_wg),
                     dim3(avg_waves(PREC) * kWave), 0, st, seg, seg64, norm, n_ppl, rho, T,
                     n_T, n_pts, f, s, out, out_a, out_v);
  return hipGetLastError();
}

template <int KIND, bool SPIN>
hipError_t launch_esc_t(const FieldArgs& f, const float* x, const float* y, int32_t n_ppl,
                        const double* rho, const double* T, int32_t n_T, int32_t n_pts,
                        const Sched& s, const uint8_t* flags, int32_t* list, int32_t* count,
                        const double* pv, const double* scale, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, st, flags, n_pts, list,
                     count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // at most n_pts points flagged: enough workgroups for the largest count
  // (the evaluation's n_items items), up to 4096 (16384 waves, 4 per SIMD on
  // 1024 SIMDs four times over)
  int64_t n_wg = (s.n_items + kWavesPerWG - 1) / kWavesPerWG;
  if (n_wg > 4096) n_wg = 4096;
  hipLaunchKernelGGL((k_escalate<KIND, SPIN>), dim3((uint32_t)n_wg), dim3(kWavesPerWG * kWave),
                     0, st, x, y, n_ppl, rho, T, n_T, n_pts, f, s, list, count, pv, scale, out);
  return hipGetLastError();
}

template <int KIND, bool SPIN, int PREC>
hipError_t launch_disc_t(const FieldArgs& f, const float4* seg, const float4* sub,
                         const double4* seg64, const double4* sub64, int32_t n_ppl,
                         const double* rho, const double* T, int32_t n_T, int32_t n_pts,
                         const Sched& s0, int32_t full, double* out, hipStream_t st) {
  if (PREC == 2 ? (sub64 == nullptr || (full && seg64 == nullptr))
                : (sub == nullptr || (full && seg == nullptr)))
    return hipErrorInvalidValue;
  Sched s = s0;
  s.n_wg = (int32_t)((s.n_items + avg_waves(PREC) - 1) / avg_waves(PREC));
  hipLaunchKernelGGL((k_disc<KIND, SPIN, PREC>), dim3(s.n_wg),
                     dim3(avg_waves(PREC) * kWave), 0, st, seg, sub, seg64, sub64, n_ppl, rho,
                     T, n_T, n_pts, f, s, full, out);
  return hipGetLastError();
}

template <int KIND, bool SPIN, int PREC>
hipError_t launch_pl_t(const FieldArgs& f, const float4* seg, const double4* seg64,
                       const float* x, const float* y, int32_t n_ppl, const SubLoop& sl,
                       const double* rho, const double* T, int32_t n_T, int32_t n_pts,
                       int64_t loop0, int64_t n_loops, double* ph, double* sp,
                       double* w, hipStream_t st) {
  if ((PREC == 2 ? seg64 == nullptr : seg == nullptr) || x == nullptr || y == nullptr)
    return hipErrorInvalidValue;
  const int32_t n_chunks = (n_pts + kWave - 1) / kWave;
  const int64_t items = n_loops * n_chunks;
  const int64_t n_wg = (items + kWavesPerWG - 1) / kWavesPerWG;
  hipLaunchKernelGGL((k_per_loop<KIND, SPIN, PREC>), dim3((uint32_t)n_wg),
                     dim3(kWavesPerWG * kWave), 0, st, seg, seg64, x, y, n_ppl, sl, rho,
                     T, n_T, n_pts, n_chunks, f, loop0, n_loops, ph, sp, w);
  return hipGetLastError();
}

#define WL_DISPATCH(FN, ...)                                                    \
  switch (f.kind * 6 + spin * 3 + precision) {                                  \
    case 0: return FN<kConst, false, 0>(__VA_ARGS__);                           \
    case 1: return FN<kConst, false, 1>(__VA_ARGS__);                           \
    case 2: return FN<kConst, false, 2>(__VA_ARGS__);                           \
    case 3: return FN<kConst, true, 0>(__VA_ARGS__);                            \
    case 4: return FN<kConst, true, 1>(__VA_ARGS__);                            \
    case 5: return FN<kConst, true, 2>(__VA_ARGS__);                            \
    case 6: return FN<kSech2, false, 0>(__VA_ARGS__);                           \
    case 7: return FN<kSech2, false, 1>(__VA_ARGS__);                           \
    case 8: return FN<kSech2, false, 2>(__VA_ARGS__);                           \
    case 9: return FN<kSech2, true, 0>(__VA_ARGS__);                            \
    case 10: return FN<kSech2, true, 1>(__VA_ARGS__);                           \
    case 11: return FN<kSech2, true, 2>(__VA_ARGS__);                           \
    case 12: return FN<kGauss, false, 0>(__VA_ARGS__);                          \
    case 13: return FN<kGauss, false, 1>(__VA_ARGS__);                          \
    case 14: return FN<kGauss, false, 2>(__VA_ARGS__);                          \
    case 15: return FN<kGauss, true, 0>(__VA_ARGS__);                           \
    case 16: return FN<kGauss, true, 1>(__VA_ARGS__);                           \
    case 17: return FN<kGauss, true, 2>(__VA_ARGS__);                           \
    case 18: return FN<kRational, false, 0>(__VA_ARGS__);                       \
    case 19: return FN<kRational, false, 1>(__VA_ARGS__);                       \
    case 20: return FN<kRational, false, 2>(__VA_ARGS__);                       \
    case 21: return FN<kRational, true, 0>(__VA_ARGS__);                        \
    case 22: return FN<kRational, true, 1>(__VA_ARGS__);                        \
    case 23: return FN<kRational, true, 2>(__VA_ARGS__);                        \
    default: return hipErrorInvalidValue;                                       \
  }

// The same over the four precisions, WL_FP32K (3) included: the launchers
// of the evaluations that offer the compensated-sum study mode.
#define WL_DISPATCH4(FN, ...)                                                   \
  switch (precision == 3 ? 24 + f.kind * 2 + spin : f.kind * 6 + spin * 3 + precision) { \
    case 24: return FN<kConst, false, 3>(__VA_ARGS__);                          \
    case 25: return FN<kConst, true, 3>(__VA_ARGS__);                           \
    case 26: return FN<kSech2, false, 3>(__VA_ARGS__);                          \
    case 27: return FN<kSech2, true, 3>(__VA_ARGS__);                           \
    case 28: return FN<kGauss, false, 3>(__VA_ARGS__);                          \
    case 29: return FN<kGauss, true, 3>(__VA_ARGS__);                           \
    case 30: return FN<kRational, false, 3>(__VA_ARGS__);                       \
    case 31: return FN<kRational, true, 3>(__VA_ARGS__);                        \
    default: WL_DISPATCH(FN, __VA_ARGS__)                                       \
  }

}  // namespace

hipError_t launch_prep(const float* d_x, const float* d_y, int64_t n_loops,
                       int32_t n_ppl, float4* d_seg, float2* d_norm, int* d_bad,
                       hipStream_t stream) {
  const int64_t total = n_loops * n_ppl;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_prep, dim3((uint32_t)blocks), dim3(256), 0, stream, d_x,
                     d_y, n_loops, n_ppl, d_seg, d_bad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // one wavefront per loop, four per workgroup
  int64_t nb = (n_loops + 3) / 4;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_norms, dim3((uint32_t)nb), dim3(256), 0, stream, d_seg, n_loops,
                     n_ppl, d_norm);
  return hipGetLastError();
}

hipError_t launch_prep64(const float* d_x, const float* d_y, int64_t n_loops,
                         int32_t n_ppl, double4* d_seg64, hipStream_t stream) {
  const int64_t total = n_loops * n_ppl;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_prep64, dim3((uint32_t)blocks), dim3(256), 0, stream, d_x, d_y,
                     n_loops, n_ppl, d_seg64);
  return hipGetLastError();
}

hipError_t launch_average(int precision, int spin, const FieldArgs& f,
                          const float4* d_seg, const double4* d_seg64, const float2* d_norm,
                          int32_t n_ppl, const double* d_rho, const double* d_T,
                          int32_t n_T, int32_t n_pts, const Sched& s, double* d_out,
                          double* d_out_a, double* d_out_v, hipStream_t stream) {
  WL_DISPATCH4(launch_avg_t, f, d_seg, d_seg64, d_norm, n_ppl, d_rho, d_T, n_T, n_pts, s,
               d_out, d_out_a, d_out_v, stream)
}

hipError_t launch_scale_escalate(int precision, int spin, const FieldArgs& f,
                                 const float* d_x, const float* d_y, int32_t n_ppl,
                                 const double* d_rho, const double* d_T, int32_t n_T,
                                 int32_t n_pts, const Sched& s, int64_t n_loops,
                                 const double* d_out_a, const double* d_out_v,
                                 double* d_scale, double* d_fp_err, uint8_t* d_flags,
                                 int32_t* d_list, double* d_out, hipStream_t stream) {
  const int64_t rows = s.n_items / s.n_chunks;  // G * n_sub
  hipLaunchKernelGGL(k_scale, dim3((uint32_t)((n_pts + 255) / 256)), dim3(256), 0, stream,
                     d_out_a, d_out_v, rows, n_pts, n_loops, (int32_t)precision, d_scale,
                     d_fp_err, d_flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || precision != 0) return e;
  switch (f.kind * 2 + spin) {
#define WL_ESC(K, SP)                                                                   \
  return launch_esc_t<K, SP>(f, d_x, d_y, n_ppl, d_rho, d_T, n_T, n_pts, s, d_flags, d_list, \
                             d_list + n_pts, d_out_v, d_scale, d_out, stream)
    case 0: WL_ESC(kConst, false);
    case 1: WL_ESC(kConst, true);
    case 2: WL_ESC(kSech2, false);
    case 3: WL_ESC(kSech2, true);
    case 4: WL_ESC(kGauss, false);
    case 5: WL_ESC(kGauss, true);
    case 6: WL_ESC(kRational, false);
    case 7: WL_ESC(kRational, true);
#undef WL_ESC
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_per_loop(int precision, int spin, const FieldArgs& f,
                           const float4* d_seg, const double4* d_seg64, const float* d_x,
                           const float* d_y, int32_t n_ppl, const SubLoop& sl,
                           const double* d_rho, const double* d_T, int32_t n_T,
                           int32_t n_pts, int64_t loop0, int64_t n_loops,
                           double* d_phase, double* d_spin, double* d_w,
                           hipStream_t stream) {
  WL_DISPATCH4(launch_pl_t, f, d_seg, d_seg64, d_x, d_y, n_ppl, sl, d_rho, d_T, n_T, n_pts,
               loop0, n_loops, d_phase, d_spin, d_w, stream)
}

hipError_t launch_prep_sub(const float* d_x, const float* d_y, int64_t n_loops,
                           int32_t n_ppl, float4* d_sub, hipStream_t stream) {
  const int64_t total = n_loops * n_ppl;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_prep_sub, dim3((uint32_t)blocks), dim3(256), 0, stream, d_x, d_y,
                     n_loops, n_ppl, d_sub);
  return hipGetLastError();
}

hipError_t launch_prep_sub64(const float* d_x, const float* d_y, int64_t n_loops,
                             int32_t n_ppl, double4* d_sub64, hipStream_t stream) {
  const int64_t total = n_loops * n_ppl;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_prep_sub64, dim3((uint32_t)blocks), dim3(256), 0, stream, d_x, d_y,
                     n_loops, n_ppl, d_sub64);
  return hipGetLastError();
}

hipError_t launch_disc(int precision, int spin, const FieldArgs& f, const float4* d_seg,
                       const float4* d_sub, const double4* d_seg64, const double4* d_sub64,
                       int32_t n_ppl, const double* d_rho, const double* d_T,
                       int32_t n_T, int32_t n_pts, const Sched& s, int32_t full,
                       double* d_out, hipStream_t stream) {
  WL_DISPATCH(launch_disc_t, f, d_seg, d_sub, d_seg64, d_sub64, n_ppl, d_rho, d_T, n_T, n_pts,
              s, full, d_out, stream)
}

hipError_t launch_disc_finish(double* d_sums, int32_t n_groups, int32_t n_pts,
                              int64_t n_loops, double* d_mean, double* d_err,
                              double* d_delta, hipStream_t stream) {
  hipLaunchKernelGGL(k_disc_finish, dim3((uint32_t)((n_pts + 255) / 256)), dim3(256), 0,
                     stream, d_sums, n_groups, n_pts, n_loops, d_mean, d_err, d_delta);
  return hipGetLastError();
}

hipError_t launch_batch(int precision, const float4* d_seg, const double4* d_seg64,
                        const float2* d_norm, const float* d_x, const float* d_y,
                        int32_t n_ppl, const void* d_hdr, int32_t n_groups, int64_t n_loops,
                        unsigned int* d_counter, double* d_res, int32_t n_wg,
                        hipStream_t stream) {
  if (precision == 2 ? d_seg64 == nullptr : d_seg == nullptr) return hipErrorInvalidValue;
  const BatchHeader* hdr = (const BatchHeader*)d_hdr;
  const int64_t lpg = n_loops / n_groups;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kBatchCounters), 0, stream, d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 blk(kWavesPerWG * kWave);
  switch (precision) {
    case 0:
      hipLaunchKernelGGL((k_batch<0>), dim3(n_wg), blk, 0, stream, d_seg, d_seg64, d_norm,
                         n_ppl, hdr, d_counter, lpg);
      break;
    case 1:
      hipLaunchKernelGGL((k_batch<1>), dim3(n_wg), blk, 0, stream, d_seg, d_seg64, d_norm,
                         n_ppl, hdr, d_counter, lpg);
      break;
    case 2:
      hipLaunchKernelGGL((k_batch<2>), dim3(n_wg), blk, 0, stream, d_seg, d_seg64, d_norm,
                         n_ppl, hdr, d_counter, lpg);
      break;
    default:
      return hipErrorInvalidValue;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scale_batch, dim3(2048), dim3(256), 0, stream, hdr, n_groups, n_loops,
                     (int32_t)precision);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (precision == 0) {
    hipLaunchKernelGGL(k_compact_batch, dim3(256), dim3(kCompactThreads), 0, stream, hdr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_esc_begin, dim3(1), dim3(1), 0, stream, hdr, n_groups, lpg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
#define WL_ESCB(K, SP, V)                                                              \
  hipLaunchKernelGGL((k_escalate_batch<K, SP>), dim3(n_wg), blk, 0, stream, d_x, d_y, n_ppl, \
                     hdr, d_counter + 1 + (V), n_groups, lpg);                          \
  if ((e = hipGetLastError()) != hipSuccess) return e;
    WL_ESCB(kConst, false, 0)
    WL_ESCB(kConst, true, 1)
    WL_ESCB(kSech2, false, 2)
    WL_ESCB(kSech2, true, 3)
    WL_ESCB(kGauss, false, 4)
    WL_ESCB(kGauss, true, 5)
    WL_ESCB(kRational, false, 6)
    WL_ESCB(kRational, true, 7)
#undef WL_ESCB
  }
  hipLaunchKernelGGL(k_reduce_batch, dim3(2048), dim3(256), 0, stream, hdr, d_res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_batch, dim3(2048), dim3(256), 0, stream, hdr, n_groups, n_loops,
                     d_res);
  return hipGetLastError();
}

hipError_t launch_reduce_sub(const double* d_partial, int32_t n_groups,
                             int32_t n_sub, int32_t n_pts, double* d_sums,
                             hipStream_t stream) {
  const int64_t total = (int64_t)n_groups * n_pts;
  hipLaunchKernelGGL(k_reduce_sub, dim3((uint32_t)((total + 255) / 256)),
                     dim3(256), 0, stream, d_partial, n_groups, n_sub, n_pts,
                     d_sums);
  return hipGetLastError();
}

hipError_t launch_stats(const double* d_sums, int32_t n_groups, int32_t n_pts,
                        int64_t n_loops, double* d_mean, double* d_err,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_stats, dim3((uint32_t)((n_pts + 255) / 256)), dim3(256),
                     0, stream, d_sums, n_groups, n_pts, n_loops, d_mean, d_err);
  return hipGetLastError();
}

}  // namespace wl
