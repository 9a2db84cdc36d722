// Internal declarations shared by the host API (wl_api.hip) and the kernels
// (wl_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wl {

// Per-segment unit-loop quantities used by the FP32 kernels, one float4 per
// segment i -> i+1 of a unit loop y (indices mod N):
//   x = m_x        = (y_i^x + y_{i+1}^x)/2       unit midpoint, x
//   y = m_y^2      = ((y_i^y + y_{i+1}^y)/2)^2   unit midpoint, y, squared
//   z = d_y        = y_{i+1}^y - y_i^y           unit step, y
//   w = c          = y_i^x y_{i+1}^y - y_i^y y_{i+1}^x   unit cross product
// so that for the scaled, shifted loop (rho_cm + s y^x, s y^y), s = sqrt(T):
//   midpoint = (rho_cm + s m_x, s m_y),   cross_i = rho_cm s d_y + T c,
// and its squared radius is (rho_cm + s m_x)^2 + T m_y^2 (m_y only enters
// squared, so the square is stored: one multiply less per segment).

// Work decomposition of one evaluation: one wavefront per item
// (group g, loop sub-range `sub`, chunk of 64 grid points).
struct Sched {
  int64_t loops_per_group;  // N_l / G
  int64_t loops_per_sub;    // ceil(loops_per_group / n_sub)
  int32_t n_sub;            // sub-ranges per group
  int32_t n_chunks;         // ceil(n_pts / 64)
  int64_t n_items;          // G * n_sub * n_chunks
  int32_t n_wg;             // workgroups (set by the launcher)
  int32_t n_xcd;            // XCDs the dispatcher round-robins over
};

// Which part of each loop a per-loop evaluation walks: segments seg_off ..
// seg_off+m-1 of the loop's N entries in the segment array passed (the
// whole-loop array, or the sub-loop one for a sub-loop), running through the
// loop's points first, first + stride, ... (mod N).  Whole loop:
// {0, N, 0, 1}; sub-loops: circle {0, N/2, 0, 2}, square {N/2, N/4, 1, 4},
// triangle {3N/4, N/4, 3, 4}.
struct SubLoop {
  int32_t seg_off, m, first, stride;
};

// Field constants prepared on the host for one launch.
struct FieldArgs {
  int32_t kind;
  // FP32 path (the sech^2 one works in scaled units with constants of its
  // own and needs none of these)
  float inv_lam2;    // 1/lambda^2
  float lam2;        // lambda^2
  float exp2_scale;  // GAUSS: -log2(e)/lambda^2
  float exp2_scale_lo, lam2_lo;  // rounding residues of exp2_scale, lam2
  float thr;         // GAUSS: rho^2 below which the polynomial branch is used
  // FP64 path
  double inv_lam_d, inv_lam2_d, lam2_d;
  // epilogue: Phi = cphi * sum_i cross_i qa_i ; S = cspin (T/N) sum_i qb_i
  // (cphi32 for the FP32 paths, whose sech^2 qa is in scaled units)
  double cphi, cspin, cphi32;
};

// Header of a batch in device memory, followed (at kBatchDescOffset) by
// n_reqs ReqDesc.  The batch kernels read the counts from here, so one
// captured launch sequence serves batches of any composition.
struct BatchHeader {
  int64_t n_reqs;
  int64_t total_items;
  int64_t total_sums;
  int64_t total_pts;
  int64_t* esc_begin;  // [8][n_reqs + 1] first FP64 recomputation item per
                       // request, per field kind x spin
};
// Work counters of a batch: the item loop, and one per field kind x spin
// for the FP64 recomputation.
constexpr int kBatchCounters = 9;
constexpr size_t kBatchDescOffset = 64;

// One request of a batched evaluation (device-resident descriptor).
struct ReqDesc {
  FieldArgs f;
  const double* rho;    // device grid
  const double* T;
  double* out;          // item outputs: partial [G*n_sub][n_pts], or the
                        // group sums directly when n_sub == 1
  double* out_a;        // [G*n_sub][n_pts] scale and rounding accumulators
  double* out_v;        //   of the items (always partial rows)
  double* scale;        // [n_pts] scale M_S of each mean
  double* fp_err;       // [n_pts] rounding-error estimate of each mean
  uint8_t* flags;       // [n_pts] grid points recomputed in FP64
  int32_t* list;        // [n_pts] the flagged points, compacted
  int32_t* count;       // [1] how many are flagged
  int64_t item_begin;   // first item of this request in the batch
  int64_t loops_per_sub;
  int64_t sums_begin;   // offset of [G][n_pts] group sums in the batch
  int64_t pts_begin;    // offset of [n_pts] means / errors in the batch
  int32_t n_sub, n_chunks, n_T, n_pts;
  int32_t spin, pad;
};

constexpr int kWavesPerWG = 4;  // batch and per-loop kernels
// k_average: waves per workgroup (barrier-coupled), by precision: 8 for
// the FP32 kernels, 4 (one per SIMD) for the FP64 ones.
constexpr int avg_waves(int prec) { return prec == 2 ? 4 : 8; }
constexpr int kWave = 64;

// Launchers (wl_kernels.hip).  All enqueue on `stream` and return the HIP
// launch status.
// Segment array d_seg of every loop (flags non-finite input in *d_bad) and
// the loop norms d_norm [n_loops] (sqrt(sum c^2), sqrt(sum d_y^2)).
hipError_t launch_prep(const float* d_x, const float* d_y, int64_t n_loops,
                       int32_t n_ppl, float4* d_seg, float2* d_norm, int* d_bad,
                       hipStream_t stream);

// d-loop generation (Sec. 2.1) into d_x, d_y [n_loops][n_ppl] (n_ppl a
// power of two, at most 8192): loops first_loop .. first_loop+n_loops-1 of
// the Philox stream keyed by `seed`.
hipError_t launch_generate(uint64_t seed, int64_t first_loop, int64_t n_loops, int32_t n_ppl,
                           float* d_x, float* d_y, hipStream_t stream);

// FP64 segment array (m_x, m_y^2, d_y, c per segment, 32 bytes) of every
// loop, used by the FP64 evaluation of whole loops.
hipError_t launch_prep64(const float* d_x, const float* d_y, int64_t n_loops,
                         int32_t n_ppl, double4* d_seg64, hipStream_t stream);

// One evaluation's main kernel: item partial sums of w into d_out, of the
// scale and rounding accumulators into d_out_a, d_out_v (all [G*n_sub]
// [n_pts]; d_out is the group sums when n_sub == 1).  d_seg (FP32 paths) or
// d_seg64 (FP64) must be set for the precision asked.
hipError_t launch_average(int precision, int spin, const FieldArgs& f,
                          const float4* d_seg, const double4* d_seg64, const float2* d_norm,
                          int32_t n_ppl, const double* d_rho, const double* d_T,
                          int32_t n_T, int32_t n_pts, const Sched& s, double* d_out,
                          double* d_out_a, double* d_out_v, hipStream_t stream);

// Per grid point from d_out_a, d_out_v: the scale (M_S), the rounding-error
// estimate of the mean and the FP64 recomputation flag (scale and fp_err
// may be NULL).  Then, for WL_FP32C, the flagged points compacted into
// d_list [n_pts + 1] (the last entry their count) and the FP64 recomputation
// of their item sums in d_out from the raw points d_x, d_y.
hipError_t launch_scale_escalate(int precision, int spin, const FieldArgs& f,
                                 const float* d_x, const float* d_y, int32_t n_ppl,
                                 const double* d_rho, const double* d_T, int32_t n_T,
                                 int32_t n_pts, const Sched& s, int64_t n_loops,
                                 const double* d_out_a, const double* d_out_v,
                                 double* d_scale, double* d_fp_err, uint8_t* d_flags,
                                 int32_t* d_list, double* d_out, hipStream_t stream);

// The segment array of the precision asked must be set: d_seg (FP32 paths)
// or d_seg64 (FP64), whole-loop or sub-loop layout as `sl` says.
hipError_t launch_per_loop(int precision, int spin, const FieldArgs& f,
                           const float4* d_seg, const double4* d_seg64, const float* d_x,
                           const float* d_y, int32_t n_ppl, const SubLoop& sl,
                           const double* d_rho, const double* d_T,
                           int32_t n_T, int32_t n_pts, int64_t loop0,
                           int64_t n_loops, double* d_phase, double* d_spin,
                           double* d_w, hipStream_t stream);

// Discretisation estimate (Sec. 4.1).  The sub-loop segment array holds,
// per loop, the N/2 segments of the circle sub-loop (points 0, 2, 4, ...),
// then the N/4 of the square one (1, 5, 9, ...) and the N/4 of the triangle
// one (3, 7, 11, ...), in the per-segment format above.
hipError_t launch_prep_sub(const float* d_x, const float* d_y, int64_t n_loops,
                           int32_t n_ppl, float4* d_sub, hipStream_t stream);
// The same sub-loop layout with the FP64 quantities of launch_prep64.
hipError_t launch_prep_sub64(const float* d_x, const float* d_y, int64_t n_loops,
                             int32_t n_ppl, double4* d_sub64, hipStream_t stream);

// Level sums for levels N, N/2, N/4: d_out [3][G*n_sub][n_pts] (with
// n_sub == 1 these are the group sums [3][G][n_pts]).  full != 0: the N
// level is the whole loop instead of the paper's combination of sub-loops.
// Sub-loops come from d_sub (FP32 paths) or d_sub64 (FP64), whole loops from
// d_seg or d_seg64; those the call uses must be set.
hipError_t launch_disc(int precision, int spin, const FieldArgs& f, const float4* d_seg,
                       const float4* d_sub, const double4* d_seg64, const double4* d_sub64,
                       int32_t n_ppl, const double* d_rho, const double* d_T,
                       int32_t n_T, int32_t n_pts, const Sched& s, int32_t full,
                       double* d_out, hipStream_t stream);

// d_sums [4][G][n_pts] with levels 0..2 filled: writes level 3 (the
// extrapolation), the means and errors [4][n_pts] and delta [n_pts] (each
// output may be NULL but d_sums).
hipError_t launch_disc_finish(double* d_sums, int32_t n_groups, int32_t n_pts,
                              int64_t n_loops, double* d_mean, double* d_err,
                              double* d_delta, hipStream_t stream);

// Batched evaluation: counter reset, persistent item kernel, scale and
// escalation flags, (WL_FP32C) persistent FP64 recomputation of the flagged
// points, sub-range reduction and statistics, all reading `d_hdr`
// (BatchHeader followed by the descriptors, whose pointers place every
// array).  Results at d_res: [group sums | means | errors | scales |
// rounding estimates | flags | ...] with the sizes from the header.  Grid
// sizes are fixed (n_wg persistent workgroups) and d_counter holds
// kBatchCounters work counters, so the sequence can be captured once and
// replayed.
hipError_t launch_batch(int precision, const float4* d_seg, const double4* d_seg64,
                        const float2* d_norm, const float* d_x, const float* d_y,
                        int32_t n_ppl, const void* d_hdr, int32_t n_groups, int64_t n_loops,
                        unsigned int* d_counter, double* d_res, int32_t n_wg,
                        hipStream_t stream);

hipError_t launch_reduce_sub(const double* d_partial, int32_t n_groups,
                             int32_t n_sub, int32_t n_pts, double* d_sums,
                             hipStream_t stream);

hipError_t launch_stats(const double* d_sums, int32_t n_groups, int32_t n_pts,
                        int64_t n_loops, double* d_mean, double* d_err,
                        hipStream_t stream);

}  // namespace wl
