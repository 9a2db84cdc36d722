/*
 * wl.h -- C ABI of the MI355X (gfx950) worldline Wilson-loop library.
 *
 * The library evaluates the loop-cloud ("worldline numerics") estimate of
 * the Wilson-loop expectation value <W(x_cm, T)> in a cylindrically
 * symmetric magnetic field B(rho) z^ (Mazur & Heyl, "Parallel Worldline
 * Numerics: Implementation and Error Analysis", arXiv:1407.7486):
 *
 *   - unit loops y(tau) of N points are scaled by sqrt(T) and moved to the
 *     centre of mass x_cm = (rho_cm, 0) (Sec. 2.1, Loop Generation);
 *   - each straight segment contributes the phase
 *       (x^i y^{i+1} - y^i x^{i+1}) * int_0^1 e A_phi(rho(t))/rho(t) dt
 *     (Sec. 3.2.1, Eqs. rhoi..Ci), evaluated with the midpoint rule;
 *   - spinors add cosh(e int_0^T B dtau) (Sec. 3.2.2, Eq. Wfermfpl);
 *   - per loop w = cos(Phi) * cosh(S)  (scalar: cos(Phi));
 *   - loops fall into G contiguous groups; the library returns the group
 *     sums of w, the mean and the standard error of the group means
 *     (Sec. 4.2.3, Grouping Worldlines), which for the mean equals the
 *     delete-a-group jackknife error.
 *
 * Conventions
 *   - Every function returns WL_OK (0) or a negative WL_E* code.  Functions
 *     taking a context store a message retrievable with wl_last_error().
 *     Nothing is printed.
 *   - A context is bound to one device and one HIP stream; it must not be
 *     used from two host threads at once.
 *   - Grid point p = j * n_T + k for rho[j], T[k]; arrays "[n_rho][n_T]" are
 *     row-major with T fastest; group sums are [G][n_rho][n_T].
 *   - Unless an argument says "device", pointers are host pointers.
 */
#ifndef WL_H
#define WL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define WL_OK 0
#define WL_EINVAL (-1)  /* invalid argument (message says which)           */
#define WL_ENOMEM (-2)  /* host or device allocation failed                */
#define WL_EHIP (-3)    /* HIP runtime error (message has the HIP string)  */
#define WL_ENODEV (-4)  /* no such device, or not a gfx950 device          */

/* ---- field kinds (Sec. 3.1, Cylindrical Magnetic Fields) --------------
 * The charge is absorbed: eB0 is e times the field on the axis, lambda
 * the tube width (ignored by WL_CONST).  With b = eB(rho) and
 * g = e A_phi(rho)/rho = e Phi_B(rho) / (2 pi rho^2):
 *   WL_CONST    b = eB0                         g = eB0/2
 *   WL_SECH2    b = eB0 sech^2(rho/lambda)      g = eB0 lambda [rho tanh(rho/
 *               lambda) - lambda ln cosh(rho/lambda)] / rho^2
 *   WL_GAUSS    b = eB0 exp(-rho^2/lambda^2)    g = eB0 lambda^2 (1 - exp(
 *               -rho^2/lambda^2)) / (2 rho^2)
 *   WL_RATIONAL the paper's validation profile f = rho^2/(lambda^2+rho^2)
 *               (Sec. 6) with flux F = eB0 lambda^2/2:
 *               b = eB0 lambda^4/(lambda^2+rho^2)^2,
 *               g = eB0 lambda^2 / (2 (lambda^2+rho^2))                    */
#define WL_CONST 0
#define WL_SECH2 1
#define WL_GAUSS 2
#define WL_RATIONAL 3

typedef struct wl_field {
  int32_t kind;     /* WL_CONST .. WL_RATIONAL                             */
  int32_t reserved; /* must be 0                                           */
  double eB0;       /* finite                                              */
  double lambda;    /* > 0 and finite for all kinds but WL_CONST           */
} wl_field;

/* ---- precision modes ---------------------------------------------------
 * WL_FP32C  FP32 segment arithmetic; phase and spin sums compensated (FP32
 *           sums over blocks of 32 segments, the block sums accumulated in
 *           FP64); FP64 per-loop epilogue and FP64 group sums.  Guarded by
 *           a rounding estimate: per-loop values whose FP32 phase may miss
 *           the phase tolerance 1e-5 max(1, |Phi|) are recomputed in FP64;
 *           for an ensemble mean whose estimated rounding error exceeds half
 *           the mean tolerance 1e-6 M_S (see wl_result), the loop
 *           sub-ranges that carry that estimate are recomputed in FP64.
 * WL_FP32   plain FP32 sums, no guard (precision-study mode).
 * WL_FP64   FP64 throughout.
 * WL_FP32K  FP32 segment arithmetic as WL_FP32C, each phase and spin sum
 *           Kahan-compensated in FP32 (sum and running compensation)
 *           instead of the block sums, FP64 epilogue and group sums, no
 *           guard: the "FP32 with compensated summation" column of the
 *           precision study (Sec. 4.3).  A precision-study mode offered by
 *           wl_average, wl_average_ex(_device), wl_average_async,
 *           wl_per_loop and wl_subloop_per_loop; the discretisation
 *           estimate, batches and the server reject it (WL_EINVAL).  The
 *           rounding estimate (fp_err) is stated as for WL_FP32C, with no
 *           recomputation.                                                   */
#define WL_FP32C 0
#define WL_FP32 1
#define WL_FP64 2
#define WL_FP32K 3

/* ---- ensemble upload flags -------------------------------------------- */
#define WL_HOST_PTR 0   /* y_x, y_y are host pointers                       */
#define WL_DEVICE_PTR 1 /* y_x, y_y are device pointers on the ctx device   */

typedef struct wl_ctx wl_ctx;
typedef struct wl_ens wl_ens;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (for example torch.cuda.current_stream().cuda_stream) or NULL for the
 * default stream; every launch and copy of this context goes to it.
 * Errors: WL_ENODEV (no such device / not gfx950), WL_ENOMEM, WL_EINVAL
 * (out == NULL). */
int wl_create(wl_ctx** out, int device, void* hip_stream);

/* Free the context and its scratch buffers (ensembles are freed with
 * wl_ensemble_free).  NULL is allowed. */
int wl_destroy(wl_ctx* ctx);

/* Message of the last failing call on ctx ("" if none).  The pointer stays
 * valid until the next call on ctx. */
const char* wl_last_error(const wl_ctx* ctx);

/* Static description of a return code. */
const char* wl_strerror(int code);

/* Library version string (static storage). */
const char* wl_version(void);

/* Ensemble upload (the device-resident loop cloud, Appendix: the loops are
 * copied to device memory once and persist across evaluations).
 * y_x, y_y: unit-loop coordinates, FP32, [n_loops][n_ppl] row-major (the
 * points of one loop contiguous), host or device memory per `flags`.  The
 * data are COPIED; the caller keeps ownership of its buffers.  The library
 * also derives per-segment quantities used by the FP32 kernels.
 * Requirements: n_loops >= 1, n_ppl >= 2, 1 <= n_groups, n_loops %
 * n_groups == 0 (equal groups, Sec. 4.2.3), all coordinates finite.
 * The call is synchronous (it returns once the copy is complete).
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_ensemble_upload(wl_ctx* ctx, const float* y_x, const float* y_y,
                       int64_t n_loops, int32_t n_ppl, int32_t n_groups,
                       int32_t flags, wl_ens** out);

/* Generate an ensemble on the device instead of uploading one: n_loops
 * d-loops of n_ppl points (a power of two, 2 .. 8192; Sec. 2.1, Loop
 * Generation, Eqs. yn2 and ynk), loops first_loop .. first_loop+n_loops-1
 * of the stream keyed by `seed`.  Random numbers: Philox4x32-10 (Salmon et
 * al., SC'11), key = seed, counter = (block, loop_lo, loop_hi, 0); uniforms
 * (w + 0.5) 2^-32; Box-Muller pairs r = sqrt(-2 ln u1),
 * (r cos 2 pi u2, r sin 2 pi u2); the new points of the recursion take the
 * pairs in order (level by level, ascending), x from the cosine and y from
 * the sine.  Each new point is the midpoint of its neighbours plus a normal
 * of standard deviation 1/sqrt(N_k); the loop's mean is subtracted.  FP64
 * arithmetic, stored as FP32.  The result is an ensemble like
 * wl_ensemble_upload's.  Synchronous.
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_ensemble_generate(wl_ctx* ctx, uint64_t seed, int64_t first_loop, int64_t n_loops,
                         int32_t n_ppl, int32_t n_groups, wl_ens** out);

/* Copy loops loop0 .. loop0+n_loops-1 of an ensemble to host arrays
 * [n_loops][n_ppl] (FP32; either pointer may be NULL).  Synchronous.
 * Errors: WL_EINVAL, WL_EHIP. */
int wl_ensemble_download(const wl_ens* ens, float* y_x, float* y_y, int64_t loop0,
                         int64_t n_loops);

/* Free an ensemble (NULL allowed).  Must be called before wl_destroy of the
 * context that created it. */
int wl_ensemble_free(wl_ens* ens);

/* Shape of an uploaded ensemble (any output pointer may be NULL). */
int wl_ensemble_info(const wl_ens* ens, int64_t* n_loops, int32_t* n_ppl,
                     int32_t* n_groups);

/* Wilson-loop ensemble average over the grid rho[n_rho] x T[n_T]
 * (Sec. 3.2 for w per loop, Sec. 4.2.3 for groups and error).
 * rho >= 0 and T > 0, all finite; spin 0 = scalar, 1 = spinor; precision
 * one of WL_FP32C, WL_FP32, WL_FP64, WL_FP32K.
 * Outputs (host, caller-owned, each may be NULL):
 *   mean       [n_rho][n_T]    (1/N_l) sum_l w_l
 *   err        [n_rho][n_T]    standard error of the group means (NaN if
 *                              G == 1); equals the delete-a-group jackknife
 *   group_sums [G][n_rho][n_T] sum of w over each group's loops, FP64
 * n_rho == 0 or n_T == 0 is an empty grid: WL_OK, nothing written.
 * Synchronous.  Results do not depend on the launch schedule: every group
 * sum has a single owner and a fixed summation order.  The first WL_FP64
 * evaluation of an ensemble (here or through the batch, server, per-loop
 * or full-loop discretisation calls) derives its FP64 segment array: 32
 * bytes per point, freed with the ensemble.
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_average(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
               const double* rho, int32_t n_rho, const double* T, int32_t n_T,
               int32_t spin, int32_t precision, double* mean, double* err,
               double* group_sums);

/* Results of an evaluation (each pointer may be NULL; see wl_average_ex).
 * With w_l = cos(Phi_l) cosh(S_l) per loop and N_l loops:
 *   mean       [n_rho][n_T]    (1/N_l) sum_l w_l
 *   err        [n_rho][n_T]    standard error of the group means
 *   group_sums [G][n_rho][n_T] sum of w over each group's loops
 *   scale      [n_rho][n_T]    M_S = (1/N_l) sum_l |w_l| max(1, S_l): the
 *                              size of the terms the mean cancels (for
 *                              scalars the mean |w|; Sec. 4.3, the fermion
 *                              problem).  M_S / |mean| is the conditioning
 *                              of the mean, and the mean's rounding
 *                              tolerance is 1e-6 M_S.
 *   fp_err     [n_rho][n_T]    estimated rounding error of the mean: from
 *                              each loop's phase-sum rounding, 32 u l_2,
 *                              l_2 = |c_Phi| sqrt(mean_i q_i^2) (T |c| +
 *                              rho_cm sqrt(T) |d_y|) over its segments (the
 *                              field weights q_i sampled every 8 segments,
 *                              |c|, |d_y| the loop's Euclidean norms of the
 *                              cross product's two parts, which are summed
 *                              apart; with even weights l_2 bounds the
 *                              parts' rounding sizes sqrt(sum_i e_i^2) of
 *                              wl_per_loop), carried to the mean
 *                              through sin(Phi) cosh(S)
 *                              and added in quadrature, plus 8 u M_S for the
 *                              roundings shared by all loops (u = 2^-24 for
 *                              the FP32 modes, 2^-53 for FP64); for a
 *                              recomputed point, that of the loop sub-ranges
 *                              left in FP32
 *   escalated  [n_rho][n_T]    1 where WL_FP32C recomputed in FP64 part of
 *                              the point (the random part of fp_err above
 *                              0.5e-6 M_S): the loop sub-ranges (G n_sub of
 *                              them) whose rounding accumulators exceed
 *                              1/(G n_sub) of the largest total that would
 *                              pass, so that the sub-ranges left in FP32
 *                              pass; else 0 */
typedef struct wl_result {
  double* mean;
  double* err;
  double* group_sums;
  double* scale;
  double* fp_err;
  uint8_t* escalated;
} wl_result;

/* wl_average with every output of wl_result.  flags WL_HOST_PTR: rho, T
 * and the outputs are host memory and the call is synchronous (as
 * wl_average); WL_DEVICE_PTR: they are device memory on the ctx device,
 * group_sums is required and the call only enqueues work on the ctx stream
 * (as wl_average_async, whose grid requirements apply).
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_average_ex(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                  const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                  int32_t spin, int32_t precision, int32_t flags, const wl_result* out);

/* As wl_average, but every array is DEVICE memory on the ctx device and
 * the call only enqueues work on the ctx stream (no host synchronisation).
 * d_rho, d_T must stay valid and unchanged until the work completes.
 * Their values are not checked on the host: a grid point with rho < 0,
 * T <= 0 or a non-finite value gets NaN in every output at that point (the
 * others are unaffected).
 * d_group_sums is required; d_mean and d_err may be NULL.  The library may
 * use its own device scratch buffer, so calls on one ctx are serialised on
 * its stream. */
int wl_average_async(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                     const double* d_rho, int32_t n_rho, const double* d_T,
                     int32_t n_T, int32_t spin, int32_t precision,
                     double* d_mean, double* d_err, double* d_group_sums);

/* Largest device scratch the allocation-free evaluation can use. */
#define WL_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* As wl_average_async, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bit for bit) as
 * wl_average_async; the call allocates nothing (no hipMalloc / hipFree, no
 * event creation) and records no kernel timing.  Its only scratch, the
 * item sums of the evaluation (w when a group's loops are split, and the
 * scale and rounding accumulators: 8 (2 or 3) G n_sub n_rho n_T bytes, n_sub
 * the library's split of each group's loops, at most 64, 1 when a group is
 * small or the grid large) and one flag byte per grid point, lives in a
 * static device array of WL_NOALLOC_SCRATCH_BYTES per device, reserved when
 * the library is loaded and held until the process ends.  Every call on a device shares that
 * array: calls that overlap on one device (two contexts or streams)
 * race and must be serialised by the caller.  Nothing in the array needs
 * to start at zero.
 * Errors: WL_EINVAL as wl_average_async, and also when the scratch would
 * exceed WL_NOALLOC_SCRATCH_BYTES (message gives both sizes) or when
 * precision is WL_FP64 and the ensemble's FP64 segment array does not exist
 * yet (an FP64 wl_average or wl_average_async derives it); WL_EHIP when the
 * scratch array's device address could not be obtained at wl_create. */
int wl_average_async_noalloc(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                             const double* d_rho, int32_t n_rho, const double* d_T,
                             int32_t n_T, int32_t spin, int32_t precision,
                             double* d_mean, double* d_err, double* d_group_sums);

/* One request of a batched evaluation (host memory, caller-owned).  The
 * outputs have the shapes of wl_average's and may each be NULL. */
typedef struct wl_request {
  wl_field field;
  const double* rho;  /* [n_rho], >= 0, finite */
  const double* T;    /* [n_T],   >  0, finite */
  int32_t n_rho;
  int32_t n_T;
  int32_t spin;       /* 0 scalar, 1 spinor */
  int32_t precision;  /* WL_FP32C, WL_FP32 or WL_FP64 */
  double* mean;       /* [n_rho][n_T] */
  double* err;        /* [n_rho][n_T] */
  double* group_sums; /* [G][n_rho][n_T] */
  double* scale;      /* [n_rho][n_T], as wl_result */
  double* fp_err;     /* [n_rho][n_T], as wl_result */
  uint8_t* escalated; /* [n_rho][n_T], as wl_result */
} wl_request;

/* Batched evaluation of n_reqs uneven requests (different fields, grids,
 * spins) against one ensemble: the work items of all requests of one
 * precision form a single index space consumed by one persistent launch
 * (Sec. 3.2 per loop, Sec. 4.2.3 groups).  Every request's result is the one
 * wl_average would return for it alone: its work is split and summed the
 * same way whatever else is in the batch.  Requests with an empty grid are
 * skipped.  Synchronous.  Validation happens for all requests before any
 * work starts (WL_EINVAL names the request).
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_average_batch(wl_ctx* ctx, const wl_ens* ens, const wl_request* reqs,
                     int32_t n_reqs);

/* ---- serving: continuous batching of requests -------------------------
 * A server evaluates submitted requests against one ensemble in batches
 * (the same arithmetic as wl_average_batch).  A scheduler thread keeps up to
 * `slots` batches in flight on streams of its own; each slot has a device
 * budget of `result_bytes` for partial sums (group sums G*n_pts*8, sub-range
 * partials G*n_sub*n_pts*8 when a group's loops are split, means and
 * errors) and `input_bytes` for descriptors and grids.  Requests are
 * admitted first-come first-served (per precision) into a free slot while
 * they fit its budget; the others wait.  Each slot's device work is one
 * captured HIP graph replayed per batch.  Each result equals wl_average's
 * for that request alone. */
typedef struct wl_server wl_server;

typedef struct wl_server_config {
  int32_t slots;       /* batches in flight, 1..8 (default 2)               */
  int32_t max_batch;   /* requests per batch (default 1024)                 */
  size_t input_bytes;  /* per slot (default 8 MiB)                          */
  size_t result_bytes; /* per slot (default 512 MiB)                        */
  int32_t in_order;    /* 0 (default): a slot's batch starts on the device
                        * as soon as it is launched, beside the previous
                        * batch (the next batch's persistent kernel takes
                        * over compute units as the previous one drains, and
                        * the previous batch's post-processing then waits
                        * for it); 1: each batch starts on the device after
                        * the previous batch has finished there (its device
                        * work is still queued ahead, so no launch gap) */
} wl_server_config;

/* Start a server on an uploaded ensemble; cfg may be NULL for defaults.
 * The ensemble and context must outlive the server.  Errors: WL_EINVAL,
 * WL_ENOMEM. */
int wl_server_create(wl_ctx* ctx, const wl_ens* ens, const wl_server_config* cfg,
                     wl_server** out);

/* Queue one request.  Its grids are copied; its output pointers are kept
 * and must stay valid until the ticket is finished.  Thread-safe.  Errors:
 * WL_EINVAL (invalid request), WL_ENOMEM (the request alone exceeds a
 * slot's budget), WL_EHIP (the server failed earlier). */
int wl_server_submit(wl_server* srv, const wl_request* req, int64_t* ticket);

/* Status of a ticket: 1 queued, 2 running, 0 done (outputs written), < 0
 * the WL_E* code it failed with.  latency_ms (may be NULL) receives the
 * time from submission to completion once finished, else -1. */
int wl_server_poll(wl_server* srv, int64_t ticket, int32_t* status, double* latency_ms);

/* Wait until the ticket finishes or timeout_s passes (< 0: no limit); then
 * as wl_server_poll. */
int wl_server_wait(wl_server* srv, int64_t ticket, double timeout_s, int32_t* status,
                   double* latency_ms);

/* Where a finished ticket's latency went: queue_ms from submission to the
 * launch of its batch, service_ms from that launch to its completion (the
 * batch's device work, the copy of its results and the hand-back; with
 * two slots the batch may share the GPU with the other slot's).  Both -1
 * while the ticket is queued or running, or if it finished without a
 * launch (an empty grid, or a failure before its batch started).
 * Returns WL_EINVAL for an unknown ticket or NULL outputs. */
int wl_server_timing(wl_server* srv, int64_t ticket, double* queue_ms, double* service_ms);

/* Forget a finished ticket. */
int wl_server_release(wl_server* srv, int64_t ticket);

/* Requests queued, requests in flight, batches launched so far. */
int wl_server_info(wl_server* srv, int64_t* pending, int64_t* running, int64_t* batches);

const char* wl_server_last_error(const wl_server* srv);

/* Finish all queued and running work, then free the server (NULL allowed). */
int wl_server_destroy(wl_server* srv);

/* Per-loop values for loops loop0 .. loop0+n_loops-1 on the grid (for
 * loop-by-loop checks).  Same kernels as wl_average.  Outputs (host, each
 * may be NULL) of shape [n_loops][n_rho][n_T]:
 *   phase     Phi in radians
 *   spin_exp  S = e int_0^T B dtau (0 is written when spin == 0)
 *   w         cos(Phi) * (spin ? cosh(S) : 1)
 * WL_FP32C: a (loop, point) whose estimated FP32 phase rounding, 32 u
 * sqrt(sum_i e_i^2), exceeds the phase tolerance 1e-5 max(1, |Phi|) is
 * recomputed in FP64 (all three values); e_i is the size of segment i's
 * rounding relative to u, (|T c_i| + |rho_cm sqrt(T) d_y,i|) q_i: the
 * cross product's two parts (Sec. 3.2.1) are summed apart, and q_i is the
 * field weight or, where the weight is the difference of two larger parts
 * (sech^2 and Gaussian beyond rho = lambda/2), the parts' size.
 * n_loops * n_rho * n_T must not exceed 2^27.
 * Synchronous.  Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_per_loop(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                int32_t spin, int32_t precision, int64_t loop0,
                int64_t n_loops, double* phase, double* spin_exp, double* w);

/* ---- discretisation estimate (Sec. 4.1, Estimating the Discretization
 * Uncertainties) ---------------------------------------------------------
 * Each loop's N points (N divisible by 4, N >= 8) form three interleaved
 * sub-loops that keep the loop's own coordinates (no re-centring):
 *   WL_SUB_CIRCLE    the N/2 points 0, 2, 4, ...
 *   WL_SUB_SQUARE    the N/4 points 1, 5, 9, ...
 *   WL_SUB_TRIANGLE  the N/4 points 3, 7, 11, ...
 * A sub-loop of M points is evaluated as a closed loop of its own: phase by
 * the midpoint rule over its M segments, spin exponent (T/M) times the sum
 * of eB over its segment midpoints.  With c, s, t the three phases and Sc,
 * Ss, St the spin exponents, each loop gives three levels of w:
 *   WL_DISC_PAPER  (the combinations the paper writes down)
 *     level N      cos(c/2 + s/4 + t/4) cosh(Sc/2 + Ss/4 + St/4)
 *     level N/2    cos(c) cosh(Sc)
 *     level N/4    cos((s + t)/2) cosh((Ss + St)/2)
 *   WL_DISC_FULL
 *     level N      the whole loop's w, as wl_average computes it
 *     level N/2    cos(c) cosh(Sc)
 *     level N/4    (cos(s) cosh(Ss) + cos(t) cosh(St)) / 2
 * (cosh factors for spinors only).  Every term of WL_DISC_FULL is a loop of
 * the discrete loop law at its own number of points, so its levels are
 * averages over N-, N/2- and N/4-point loops; the paper's N and N/4 levels
 * average correlated sub-loop phases instead, which narrows the phase
 * distribution (for a constant field both lie above the finite-N averages).
 * WL_DISC_PAPER walks each loop's N sub-loop segments once; WL_DISC_FULL
 * walks the whole loop as well (twice the segment work).
 * Level 3 is the parabola in 1/N through the three levels, evaluated at
 * 1/N = 0: 8/3 W_N - 2 W_{N/2} + 1/3 W_{N/4}, formed group by group so that
 * its error is the standard error of its group means; delta = |W_N - W_inf|
 * is the paper's estimate of the discretisation uncertainty. */
#define WL_DISC_PAPER 0
#define WL_DISC_FULL 1

#define WL_SUB_CIRCLE 0
#define WL_SUB_SQUARE 1
#define WL_SUB_TRIANGLE 2

/* Discretisation estimate over the grid rho[n_rho] x T[n_T] (arguments as
 * wl_average; mode WL_DISC_PAPER or WL_DISC_FULL).  Outputs (host,
 * caller-owned, each may be NULL), levels in the order N, N/2, N/4,
 * extrapolated:
 *   mean       [4][n_rho][n_T]
 *   err        [4][n_rho][n_T]     standard error of the group means
 *   delta      [n_rho][n_T]        |mean[0] - mean[3]|
 *   group_sums [4][G][n_rho][n_T]
 * The first call with WL_FP32C or WL_FP32 on an ensemble derives its
 * sub-loop segment array (16 bytes per point), the first with WL_FP64 its
 * FP64 sub-loop segment array (32 bytes per point); both are freed with
 * the ensemble.
 * Synchronous; deterministic like wl_average.  Errors: WL_EINVAL (also for
 * n_ppl not divisible by 4 or below 8), WL_ENOMEM, WL_EHIP. */
int wl_discretisation(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                      const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                      int32_t spin, int32_t precision, int32_t mode, double* mean,
                      double* err, double* delta, double* group_sums);

/* As wl_per_loop, for one sub-loop (WL_SUB_*) of each loop: phase,
 * spin exponent (T/M) sum eB and w of that sub-loop alone.  Same kernels
 * and sub-loop data as wl_discretisation. */
int wl_subloop_per_loop(wl_ctx* ctx, const wl_ens* ens, const wl_field* field,
                        const double* rho, int32_t n_rho, const double* T, int32_t n_T,
                        int32_t spin, int32_t precision, int32_t subloop, int64_t loop0,
                        int64_t n_loops, double* phase, double* spin_exp, double* w);

/* ---- effective action (Eq. cylEA; Sec. 3.3, Renormalization; Sec. 6,
 * Implementation) --------------------------------------------------------
 * From the group sums of an evaluation on the grids of wl_action_grids, per
 * group g with W_g = G S_g / N_l and eB = eB(rho_cm):
 *   integrand  I(T) = e^{-m^2 T} / T^3 [W_g - 1 - (eB T)^2 / 3]   (spinor)
 *              I(T) = e^{-m^2 T} / T^3 [W_g - 1 + (eB T)^2 / 6]   (scalar)
 *   density    D_g(rho) = int_0^a (small-T series of I, Eqs. fermI and
 *              scalI, to T^4) dT + int_a^inf I dT, the latter by Simpson's
 *              rule on n_T uniform intervals of x = 1/(1 + T/T_max)
 *   action     (1/4pi) int_0^inf rho D_g(rho) drho by Simpson's rule on
 *              n_rho uniform intervals of x = 1/(1 + rho/rho_max) (per unit
 *              time and length along the field; NaN for WL_CONST, whose
 *              action diverges)
 * and the mean and standard error over the groups (the integrals are done
 * group by group, Sec. 4.2.3).  The LCF comparison (Sec. 6) is the same
 * integral with W replaced by the constant-field form at eB(rho_cm):
 * eB T coth(eB T) (spinor) or eB T / sinh(eB T) (scalar).  The scalar case
 * uses the same measure (1/4pi) rho drho. */
typedef struct wl_action_spec {
  double m2;      /* mass squared, > 0 (units of eB)                        */
  double a;       /* small-T cut: the series is used below a, > 0           */
  double T_max;   /* scale of the T substitution, > 0                       */
  double rho_max; /* scale of the rho substitution, > 0                     */
  int32_t n_T;    /* Simpson intervals in T (even, >= 2) = T grid points    */
  int32_t n_rho;  /* Simpson intervals in rho (even, >= 2) = rho grid points*/
} wl_action_spec;

/* Output pointers of wl_action; each may be NULL. */
typedef struct wl_action_out {
  double* density;      /* [G][n_rho] per group                             */
  double* density_mean; /* [n_rho]                                          */
  double* density_err;  /* [n_rho] standard error of the group densities    */
  double* action;       /* [G]                                              */
  double* action_mean;  /* [1]                                              */
  double* action_err;   /* [1]                                              */
  double* lcf_density;  /* [n_rho]                                         */
  double* lcf_action;   /* [1]                                              */
} wl_action_out;

/* The grids the action integrals need: T[n_T] ascending with T[0] = a
 * (x_k = k x_a / n_T, x_a = 1/(1 + a/T_max), k = n_T .. 1) and
 * rho[n_rho] ascending with rho[0] = 0 (x_k = k / n_rho); the node x = 0
 * (infinity) contributes nothing.  Host arrays.  Errors: WL_EINVAL. */
int wl_action_grids(const wl_action_spec* spec, double* T, double* rho);

/* Effective action from group sums [G][n_rho][n_T] evaluated on those grids
 * (for example wl_average's, G = n_groups of an ensemble of n_loops loops)
 * for the given field and spin.  flags WL_HOST_PTR: group_sums and the
 * outputs are host memory; WL_DEVICE_PTR: device memory on the ctx device.
 * Synchronous in both cases.  Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_action(wl_ctx* ctx, const wl_action_spec* spec, const wl_field* field,
              int32_t spin, const double* group_sums, int32_t n_groups, int64_t n_loops,
              int32_t flags, const wl_action_out* out);

/* ---- correlations between grid points and group reassignment (Sec. 4.2,
 * Eq. corrcoef; Sec. 4.2.3, Grouping Worldlines) --------------------------
 * Per-loop values come from an evaluation with one loop per group (see
 * wl_ensemble_set_groups): its group sums [N_l][n_rho][n_T] are the w of
 * each loop at each grid point. */

/* Change the number of contiguous groups of an ensemble (1 <= n_groups,
 * n_groups divides n_loops); later evaluations use it.  Not while a server
 * (wl_server_create) runs on the ensemble or work on it is in flight.
 * Errors: WL_EINVAL. */
int wl_ensemble_set_groups(wl_ens* ens, int32_t n_groups);

/* Correlation coefficients between the n_pts columns of values [n_units]
 * [n_pts] (per-loop w, or group sums, at each grid point) over the n_units
 * rows: corr[p][q] = sum_k (x_kp - m_p)(x_kq - m_q) / sqrt(S_p S_q), m the
 * column means and S_p = sum_k (x_kp - m_p)^2 (NaN for a constant column).
 * corr is [n_pts][n_pts], exactly symmetric.  The Gram matrix runs on the
 * FP64 matrix cores; deterministic.  flags WL_HOST_PTR: values and corr are
 * host memory, WL_DEVICE_PTR: device memory.  n_units >= 2,
 * 1 <= n_pts <= 16384.  Synchronous.  Errors: WL_EINVAL, WL_ENOMEM,
 * WL_EHIP. */
int wl_correlation(wl_ctx* ctx, const double* values, int64_t n_units, int32_t n_pts,
                   int32_t flags, double* corr);

/* Group sums under a reassignment of the units (loops) to groups:
 * sums[g][p] = sum_{j < n_units/n_groups} per_unit[perm[g n_units/n_groups
 * + j]][p], where perm is row point_perm[p] of perms [n_perms][n_units]
 * (row 0 for every point if point_perm is NULL).  Independent random rows
 * for different grid points give the paper's shuffled groups.  Each row of
 * perms must be a permutation of 0 .. n_units-1 and n_groups must divide
 * n_units.  flags as wl_correlation (all arrays host or all device); host
 * arrays are validated, device ones are only range-checked (WL_EINVAL after
 * the fact, out-of-range entries skipped).  Synchronous.
 * Errors: WL_EINVAL, WL_ENOMEM, WL_EHIP. */
int wl_regroup(wl_ctx* ctx, const double* per_unit, int64_t n_units, int32_t n_pts,
               const int64_t* perms, int32_t n_perms, const int32_t* point_perm,
               int32_t n_groups, int32_t flags, double* sums);

/* Kernel timing: when enabled, the main evaluation kernel of each
 * wl_average / wl_average_async / wl_discretisation call, the generation
 * kernels of wl_ensemble_generate and the Gram kernel of wl_correlation are
 * bracketed by HIP events on the ctx stream.  wl_set_timing(ctx, 1) also forgets earlier records.
 * wl_last_kernel_ms waits for the last recorded launch and returns its
 * duration in milliseconds; wl_kernel_ms_total waits for all of them and
 * returns the sum of their durations and their count.  Both return
 * WL_EINVAL if nothing was recorded. */
int wl_set_timing(wl_ctx* ctx, int32_t enable);
int wl_last_kernel_ms(wl_ctx* ctx, double* ms);
int wl_kernel_ms_total(wl_ctx* ctx, double* total_ms, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* WL_H */
