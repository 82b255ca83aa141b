/*
 * bf.h -- C ABI of libbf.so, the MI355X (gfx950) implementation of the
 * accelerated shiftable O(1) Gaussian bilateral filter (Chaudhury,
 * "Acceleration of the shiftable O(1) algorithm for bilateral filtering and
 * non-local means").
 *
 * The filter computed is Algorithm 2 of the paper:
 *   1. window radius R (a factor of sigma_s, Section 2: R = 3 sigma_s),
 *   2. the dynamic range T of eq. (bound) by Algorithm 1 (row then column
 *      MAX-FILTER of the Appendix) or a caller-given global T,
 *   3. the order N = 0.405 (T/sigma_r)^2 (Section 1.3, Table 1),
 *   4. the truncation M by the sigma_r bands of Algorithm 2 step 4 with eqs.
 *      (trunc) and (Chernoff),
 *   5. the truncated raised-cosine range kernel of eq. (approx),
 *   6. SHIFTABLE-BF (Section 1.2): for every kept frequency the images
 *      f cos(w f), f sin(w f), cos(w f), sin(w f) are smoothed by a separable
 *      spatial Gaussian (eq. (GF)) and combined by eqs. (f1), (f2).
 *
 * Conventions shared by every entry point:
 *  - Every function returns bf_status; nothing throws across the ABI.
 *  - Device pointers are HIP device addresses on the current device; the
 *    caller owns them and keeps them alive until the stream work completes.
 *  - `hip_stream` is a hipStream_t (NULL = the null stream).  All device work
 *    of a call is enqueued on it; calls return without synchronising unless a
 *    report is requested.
 *  - All argument checks run before any launch: a call that returns an error
 *    has enqueued no work and written no output.
 *  - Images are row-major, `in_pitch`/`out_pitch` elements between rows.
 *    Input: uint8, uint16 or float32.  Output: always float32, same units as
 *    the input.
 *  - A plan is not re-entrant: one stream at a time per plan.  Separate plans
 *    on separate streams are independent.
 *
 * Environment (read at plan creation; results stay within the same error
 * bar, only launch shapes and timing change):
 *  - BF_TUNE_CACHE=<file>: the autotuner's choices are read from and
 *    appended to this file (one JSON object per line); BF_TUNE_LOG prints
 *    them to stderr.
 *  - BF_GRAPH=0: launch the kernels directly instead of replaying a captured
 *    HIP graph.
 *  - BF_Z_BUDGET_MB=<n>: device memory for the smoothed images of a launch
 *    (default 64 GiB); a smaller budget runs the pairs in several launches,
 *    and a batch whose images need more runs them one after another.
 *  - Shape overrides for measurement: BF_HCHUNK / BF_VCHUNK (16 or 32
 *    samples per thread of the recursive passes), BF_H_WG / BF_V_WG
 *    (workgroups the recursive passes aim for), BF_TOEP_LDS_KB (LDS of a
 *    Toeplitz workgroup).
 *  - BF_FAIL_ALLOC: every device allocation fails with BF_ERR_OUT_OF_MEMORY
 *    (a test hook for that path).
 */
#ifndef BF_H_
#define BF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = 1,   /* a parameter is out of its documented range     */
  BF_ERR_UNSUPPORTED = 2,   /* valid but beyond the library's limits          */
  BF_ERR_OUT_OF_MEMORY = 3, /* a device or host allocation failed             */
  BF_ERR_DEVICE = 4,        /* a HIP call failed (see bf_last_error_detail)   */
  BF_ERR_NOT_FINITE = 5,    /* float input held NaN or Inf (report requested) */
  BF_ERR_RANGE = 6          /* input exceeded value_range (report requested)  */
} bf_status;

typedef enum { BF_U8 = 0, BF_U16 = 1, BF_F32 = 2 } bf_dtype;

/* How T is obtained (Algorithm 2 step 2). */
typedef enum {
  BF_T_GLOBAL = 0, /* T = t_value (0 => value_range), as in the original SHIFTABLE-BF */
  BF_T_LOCAL = 1   /* T from Algorithm 1 over the (2R+1)^2 square window          */
} bf_trange;

/* Implementation of the spatial smoothing of SHIFTABLE-BF step 3.  Each
 * variant implements one discrete spatial operator (see bf_spatial). */
typedef enum {
  BF_BLUR_AUTO = 0,            /* autotuner picks among the implementations of the
                                  operator bf_params.spatial names that meet the error
                                  gate; it never changes the operator itself             */
  BF_BLUR_IIR_F32 = 1,         /* Young-van Vliet recursive Gaussian, FP32 scans          */
  BF_BLUR_TOEPLITZ_F16 = 2,    /* FIR taps exp(-j^2/2 s^2), |j|<=R, FP16 MFMA, FP32 acc   */
  BF_BLUR_TOEPLITZ_BF16 = 3,   /* same FIR, BF16 MFMA, FP32 accumulation                  */
  BF_BLUR_TOEPLITZ_F16X2 = 4,  /* same FIR, FP16 hi+lo split operands, FP32 accumulation  */
  BF_BLUR_TOEPLITZ_BF16X2 = 5  /* same FIR, BF16 hi+lo split operands, FP32 accumulation  */
} bf_blur;

/* Spatial kernel of eq. (BF) (the filter smoothed by step 3).  The paper
 * leaves the discrete O(1) smoother open (Section 1.2); the operator is fixed
 * by this field and by nothing else, so equal parameters give equal images
 * whatever the autotuner picks. */
typedef enum {
  BF_SPATIAL_GAUSSIAN = 0,     /* Gaussian of sigma_s.  With BF_BLUR_IIR_F32 or
                                  BF_BLUR_AUTO: the recursive Young-van Vliet filter.
                                  With a Toeplitz variant: the sampled FIR below (the
                                  variant names the operator).                          */
  BF_SPATIAL_BOX = 1,          /* constant filter over the (2R+1)^2 square (Section 4, the
                                  comparison with integral histograms); R = radius, or
                                  round(sigma_s) when radius is 0.  Toeplitz variants only
                                  (unit taps).                                           */
  BF_SPATIAL_GAUSSIAN_FIR = 2  /* sampled Gaussian taps exp(-j^2/2 sigma_s^2), |j| <= R.
                                  Toeplitz variants only; BF_BLUR_AUTO picks among them. */
} bf_spatial;

/* Range kernel of SHIFTABLE-BF (Section 1.2).  Both tend to the Gaussian of
 * sigma_r (Section 1.3). */
typedef enum {
  BF_RANGE_RAISED_COSINE = 0,  /* eq. (RC): cos^N(s / (sqrt(N) sigma_r)), N from T (Table 1
                                  rule), truncated by Algorithm 2 step 4                  */
  BF_RANGE_POLYNOMIAL = 1      /* eq. (RPconv): (1 - s^2 / (2 N sigma_r^2))^N with the
                                  smallest N >= 0.5 (T/sigma_r)^2, expanded in Chebyshev
                                  polynomials of the intensity over [0, value_range]; the
                                  orders whose summed coefficient bound is <= eps dropped.
                                  8-bit input and global T only; plans whose FP32 sums
                                  would cancel (T far below value_range) are refused.    */
} bf_range_kernel;

typedef struct {
  int32_t height, width;   /* >= 1                                                   */
  int64_t in_pitch;        /* elements between input rows; 0 => width               */
  int64_t out_pitch;       /* elements between output rows; 0 => width              */
  bf_dtype dtype;
  double sigma_s;          /* spatial sigma in pixels (> 0; >= 0.5 for the IIR)     */
  double sigma_r;          /* range sigma in intensity units (> 0)                  */
  double eps;              /* truncation tolerance, 0 < eps < 1 (fraction of peak)  */
  int32_t radius;          /* window R, 0 => ceil(3 sigma_s); also the FIR radius   */
  bf_trange t_mode;
  double t_value;          /* GLOBAL only: T; 0 => value_range                      */
  double value_range;      /* intensities lie in [0, value_range]; 0 => 255 for u8
                              and f32, 65535 for u16.  Sets the T table size and
                              the sigma_r bands (given in 8-bit units) of step 4. */
  bf_blur blur;
  bf_spatial spatial;
  bf_range_kernel range_kernel;
  /* Non-local means (the paper's closing section, eqs. (NL1), (NL2)): with
   * patch_size p >= 2 the range kernel compares the patches u_1 = (0, 0),
   * u_k = (patch_dy[k-1], patch_dx[k-1]) (k = 2..p, |offsets| <= 2) of the
   * output pixel and of each neighbour: the product of p raised cosines of
   * sigma_r, each of order N and truncation M from T as for the bilateral
   * filter, expanded into one term per multi-index of kept frequencies.
   * Patch samples outside the image take the nearest pixel.  8-bit input,
   * the raised-cosine kernel and the Toeplitz split variants only
   * (BF_BLUR_TOEPLITZ_F16X2 / BF16X2; the box spatial filter gives eq. (NL1)
   * as written).  0 or 1: the bilateral filter.  patch_dy[0], patch_dx[0]
   * must be 0. */
  int32_t patch_size;
  int32_t patch_dy[4], patch_dx[4];
} bf_params;

/* Per-image result summary (filled only when requested; requesting it makes
 * the call synchronise its stream). */
typedef struct {
  double T;          /* dynamic range used (raw maximum for float input)      */
  int32_t T_used;    /* integer T indexing the order table (ceil for floats)   */
  int32_t N, M;      /* order and truncation (polynomial kernel: M = highest
                        kept Chebyshev order J)                                */
  int32_t kept;      /* kept terms N - 2M + 1 (polynomial kernel: J + 1; per
                        patch sample for non-local means)                      */
  int32_t pairs;     /* frequency pairs blurred (with the zero frequency; for
                        non-local means the folded multi-indices)              */
  int32_t variant;   /* bf_blur actually run                                   */
  int32_t flags;     /* bit0 non-finite input, bit1 T above value_range        */
  int64_t q_nonpos;  /* pixels whose denominator (f2) was <= 0 (output = input) */
  float ms;          /* device time of the call                                */
} bf_report;

typedef struct bf_plan_s *bf_plan_t;

/* Build a plan for n_images images; params[i] describes image i.  Host-side
 * FP64 order/coefficient tables for every integer T in [0, value_range] and
 * the operator constants are computed and uploaded; the workspace is
 * allocated on the current device.  No image data is read.
 * Errors: BF_ERR_INVALID_ARG (bad params, n_images < 1, NULL pointers),
 * BF_ERR_UNSUPPORTED (order beyond the build limits; width or height above
 * 8192 for the recursive blur; radius above 120 for the Toeplitz blur; the
 * box or sampled-FIR spatial filter with the recursive blur),
 * BF_ERR_OUT_OF_MEMORY, BF_ERR_DEVICE.  On error *out is set to NULL. */
bf_status bf_plan(const bf_params *params, int32_t n_images, bf_plan_t *out);

/* Filter image 0 of the plan: d_in (dtype, in_pitch) -> d_out (float32,
 * out_pitch).  Enqueued on hip_stream; rep (nullable) receives the summary and
 * makes the call synchronise.  BF_ERR_NOT_FINITE / BF_ERR_RANGE can only be
 * returned when rep is given (they need the device flags). */
bf_status bf_filter(bf_plan_t plan, const void *d_in, float *d_out, void *hip_stream,
                    bf_report *rep);

/* Filter images 0..n-1 of the plan (n <= n_images) in one graph launch of the
 * batched kernels: d_in[i] / d_out[i] are device pointers to image i (host
 * arrays of n pointers).  reps (nullable) has n entries. */
bf_status bf_filter_batch(bf_plan_t plan, int32_t n, const void *const *d_in, float *const *d_out,
                          void *hip_stream, bf_report *reps);

/* bf_filter for callers that cannot allocate device memory during the call:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Filters image 0 of the plan with the same kernels and tables as
 * bf_filter; the working memory (device state, row maxima, cos/sin tables,
 * partial sums, smoothed images) comes from a static array of 256 MiB per
 * device that the library holds until the process ends, not from the plan.
 * The call launches its kernels directly on hip_stream (no graph of its own,
 * so a caller may capture it) and calls no hipMalloc, hipFree or other
 * allocating routine.  The frequency pairs run in as many launches as the
 * 256 MiB need (one for images up to about 0.5 megapixels at 40 pairs).
 * Every call on one device shares that device's array: calls that overlap on
 * one GPU (any plan, any stream) race and give undefined results; callers
 * serialise them.  rep (nullable) makes the call synchronise its stream, so
 * pass NULL under capture.
 * Errors: as bf_filter; BF_ERR_UNSUPPORTED when the working memory of one
 * pair per launch exceeds 256 MiB (about 10 megapixels on the recursive
 * blur); BF_ERR_INVALID_ARG when the current device is not the one the plan
 * was made on. */
bf_status bf_filter_noalloc(bf_plan_t plan, const void *d_in, float *d_out, void *hip_stream, bf_report *rep);

/* Algorithm 1 alone for image 0: writes the dynamic range T (raw, before any
 * ceil) to *T_out after synchronising hip_stream. */
bf_status bf_dynamic_range(bf_plan_t plan, const void *d_in, void *hip_stream, double *T_out);

/* Stage timing.  While enabled, every filter call of the plan records HIP
 * events on its stream between the stages it launches (range; vertical pass
 * of the recursive blur; vertical pass of the Toeplitz blur; horizontal pass +
 * combine of either, with the sum of the pair groups).  bf_profile_read
 * synchronises the plan's last stream, returns the summed device milliseconds
 * and launch counts per stage since the last read, and clears them.  Stage
 * indices are the BF_STAGE_* values. */
enum {
  BF_STAGE_RANGE = 0,
  BF_STAGE_V_IIR = 1,
  BF_STAGE_V_TOEPLITZ = 2,
  BF_STAGE_H_COMBINE = 3,
  BF_STAGE_COUNT = 4
};
bf_status bf_profile(bf_plan_t plan, int32_t enable);
bf_status bf_profile_read(bf_plan_t plan, double *ms /* [BF_STAGE_COUNT] */,
                          int64_t *launches /* [BF_STAGE_COUNT] */);

/* Release the plan.  The caller synchronises the plan's streams first. */
void bf_plan_destroy(bf_plan_t plan);

/* Static description of a status code. */
const char *bf_status_string(bf_status s);

/* Detail of the last BF_ERR_DEVICE / BF_ERR_UNSUPPORTED on this thread. */
const char *bf_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* BF_H_ */
