/*
 * ssimx.h -- C-ABI of the MI355X (gfx950) SSIM / MS-SSIM library.
 *
 * Operations follow "A Hitchhiker's Guide to Structural Similarity"
 * (Venkataramanan et al., arXiv 2101.06354):
 *   - local statistics, luminance / contrast-structure terms and the quality
 *     map: Background section, equations local_means .. local_corr, lum_term,
 *     the cs form with C3 = C2/2, and the mean-SSIM pooling;
 *   - C1 = (K1 L)^2, C2 = (K2 L)^2: Background section;
 *   - rectangular windows through window sums / integral images:
 *     Performance-Efficiency subsection, equations integral_image_start ..
 *     corr_from_sum;
 *   - stride: "Effect of stride" subsection;
 *   - border handling (valid / zero / reflection): table of implementation
 *     features (tab:ssim_implementation_details);
 *   - MS-SSIM with 2x2 average-pooling pyramids, cs at every scale, luminance
 *     at the coarsest, exponentially weighted product and exponent
 *     renormalisation when fewer scales are used: Introduction and the
 *     MS-SSIM implementation list of the "Versions of SSIM" section.
 * The backward calls are the adjoint of those definitions with respect to the
 * distorted plane (the paper mentions MS-SSIM as a training objective only).
 *
 * Conventions shared by every call:
 *   - All data pointers are DEVICE pointers unless the comment says "host".
 *     The caller owns every buffer (inputs, outputs, workspace).  Compute
 *     calls allocate no device memory.  Only a batch plan owns memory, which
 *     ssimx_plan_destroy releases.
 *   - `stream` is a hipStream_t handle passed as void* (NULL = the null
 *     stream).  Compute calls are asynchronous on it; results are valid after
 *     the stream has been synchronised.
 *   - Planes are row-major.  `pitch` = elements between rows (>= width),
 *     `batch_stride` = elements between frames.  Planes of one call all have
 *     the same width and height.
 *   - Argument errors are detected on the host before any launch and return
 *     a negative ssimx_status; nothing is launched then.  Launch limits are
 *     argument errors too: a call takes 1..65535 frames (`batch`, `frames`;
 *     1..21845 RGB frames for ssimx_color_ssim, whose three channels are
 *     launched as frames), and a plane holds at most 2^31 - 2^16 pixels;
 *     beyond either, SSIMX_EINVAL.  A failed launch
 *     returns SSIMX_EHIP and ssimx_last_hip_error() gives the hipError_t.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *   - NaN/Inf in inputs propagate to outputs.
 *   - Map outputs are float32, of size map_shape().  Accumulation is float32;
 *     pooled scores use a fixed-order compensated reduction (deterministic).
 */
#ifndef SSIMX_H
#define SSIMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSIMX_VERSION 101

typedef enum {
  SSIMX_OK = 0,
  SSIMX_EINVAL = -1,     /* bad argument (null pointer, k < 1, even Gaussian k, sigma <= 0, stride < 1, C1/C2 < 0, ...) */
  SSIMX_EDTYPE = -2,     /* unsupported dtype for this operation */
  SSIMX_ETOOSMALL = -3,  /* map would be empty, or an MS-SSIM scale is smaller than the window */
  SSIMX_EWORKSPACE = -4, /* ws is NULL or ws_bytes below ssimx_workspace_size() */
  SSIMX_EHIP = -5,       /* a HIP runtime call failed; see ssimx_last_hip_error() */
  SSIMX_ENOTSUP = -6,    /* valid but unsupported combination */
  SSIMX_ENOMEM = -7,     /* plan creation could not allocate */
  SSIMX_ESCRATCH = -8    /* ssim_pooled_noalloc: the call needs more scratch than
                            its static per-device buffer holds */
} ssimx_status;

typedef enum { SSIMX_U8 = 0, SSIMX_U16 = 1, SSIMX_F32 = 2, SSIMX_BF16 = 3 } ssimx_dtype;

/* Window shape (Background section): Gaussian taps g_t ~ exp(-(t-c)^2 /
 * (2 sigma^2)), c = (k-1)/2, normalised to sum 1, 2-D weight g_m g_n; or the
 * rectangular window with weight 1/k^2. */
typedef enum { SSIMX_WIN_GAUSSIAN = 0, SSIMX_WIN_BOX = 1 } ssimx_window;

/* Rectangular windows on integer planes: AUTO/SEPARABLE = tile-local exact
 * integer window sums; INTEGRAL_IMAGE = the paper's five summed-area tables
 * (uint32, wrap-around) and the four-corner formula.  Both give the same
 * integer sums where INTEGRAL_IMAGE is accepted: 8-bit planes (k <= 64 keeps
 * every window sum below 2^32).  For 16-bit planes a window sum of squares
 * reaches 2^32 from k = 2 (k^2 * 65535^2), which uint32 tables cannot hold,
 * so INTEGRAL_IMAGE with uint16 and k > 1 returns SSIMX_ENOTSUP (AUTO gives
 * the exact sums).  Ignored for Gaussian windows. */
typedef enum { SSIMX_ALGO_AUTO = 0, SSIMX_ALGO_SEPARABLE = 1, SSIMX_ALGO_INTEGRAL_IMAGE = 2 } ssimx_algo;

/* VALID: windows fully inside the plane.  ZERO / REFLECT: the plane is
 * extended by floor((k-1)/2) before and ceil((k-1)/2) after, with zeros or by
 * half-sample symmetric reflection (x[-1] = x[0]). */
typedef enum { SSIMX_PAD_VALID = 0, SSIMX_PAD_ZERO = 1, SSIMX_PAD_REFLECT = 2 } ssimx_pad;

typedef struct {
  int window;    /* ssimx_window */
  int k;         /* window size, 1..41 for Gaussian (odd), 1..64 for box */
  float sigma;   /* Gaussian standard deviation (> 0); ignored for box */
  double C1;     /* (K1 L)^2 >= 0 */
  double C2;     /* (K2 L)^2 >= 0 */
  int stride;    /* >= 1; windows anchored at (stride*i, stride*j) */
  int padding;   /* ssimx_pad */
  int algo;      /* ssimx_algo */
} ssimx_params;

typedef struct {
  const void* data;     /* device pointer to frame 0, row 0 */
  int dtype;            /* ssimx_dtype */
  int width, height;
  int64_t pitch;        /* elements between rows */
  int64_t batch_stride; /* elements between frames */
} ssimx_image;

/* MS-SSIM flags. */
#define SSIMX_MS_RENORM 1   /* divide the n_scales weights by their sum */
#define SSIMX_MS_CS_CLAMP 2 /* use max(CS_j, 0) (and max(S_M, 0)); default lets a
                               negative value with a fractional exponent give NaN */
#define SSIMX_MS_SUM 4      /* 'Sum' aggregation (Versions of SSIM section; the
                               Scikit-Video notes of the Implementations section):
                               score = sum_j w_j T_j over the same terms T_j (CS_j,
                               j < M; S_M) with the weights divided by their sum
                               (implies RENORM; CS_CLAMP has no effect).
                               Other flag bits: EINVAL.  RENORM or SUM with
                               weights summing to zero: EINVAL. */
#define SSIMX_MS_COARSE_SEPARATE 8 /* coarsest term mean(l) * mean(cs) instead of
                               the default mean(l * cs) (the paper describes the
                               combination without printing it; both readings
                               are offered).  Supported by msssim,
                               msssim_backward and ssimx_msssim3d. */

/* Operation selector for ssimx_workspace_size(). */
typedef enum {
  SSIMX_OP_MAP = 0, SSIMX_OP_POOLED = 1, SSIMX_OP_MSSSIM = 2,
  SSIMX_OP_MAP_BACKWARD = 3, SSIMX_OP_POOLED_BACKWARD = 4, SSIMX_OP_MSSSIM_BACKWARD = 5
} ssimx_op;

/* Host only.  Map size: floor((H' - k)/stride) + 1 per axis with H' = H
 * (valid) or H + k - 1 (zero, reflect).  Returns ETOOSMALL when empty. */
ssimx_status ssimx_map_shape(const ssimx_params* p, int width, int height, int* width_out, int* height_out);

/* Host only.  Device workspace bytes needed by `op` for `batch` frames of
 * width x height (n_scales is used by the MS-SSIM ops only). */
ssimx_status ssimx_workspace_size(const ssimx_params* p, int op, int dtype, int width, int height,
                                  int batch, int n_scales, size_t* bytes);

/* SSIM quality map Q(i,j) = l * cs of each frame pair (Background section).
 * map_out: float32 [batch][map_h][map_pitch] with frame stride
 * map_batch_stride (elements).  score_out (nullable): float32 [batch] mean of
 * each map.  ref and dis must have equal sizes and dtypes. */
ssimx_status ssim_map(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                      float* map_out, int64_t map_pitch, int64_t map_batch_stride, float* score_out,
                      void* ws, size_t ws_bytes, void* stream);

/* Mean SSIM per frame pair, without writing the map.  score_out: float32 [batch]. */
ssimx_status ssim_pooled(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                         float* score_out, void* ws, size_t ws_bytes, void* stream);

/* Luminance-Weighted Pooling subsection: score_out[b] = (1 / map positions)
 * sum w(mu_1) Q over the map, mu_1 the reference's local mean (float32, from
 * the same statistics as Q), w = 0 for mu_1 < a_s, (mu_1 - a_s) / b_s on
 * [a_s, a_s + b_s), 1 from a_s + b_s on (b_s = 0: a step at a_s, decided in
 * float32).  The weighted sum is divided by the number of positions, not by
 * the sum of the weights; a_s = b_s = 0 gives ssim_pooled's score for
 * non-negative planes.  a_s, b_s finite, b_s >= 0 (else EINVAL).  Only the
 * stride-1 Gaussian windows of the fast path (k = 7, 9, 11, 13, centre taps
 * >= 0.04; any padding) are supported, else ENOTSUP.  Workspace: as
 * ssim_pooled. */
ssimx_status ssim_pooled_lw(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                            float a_s, float b_s, float* score_out, void* ws, size_t ws_bytes, void* stream);

/* ssim_pooled for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same scores as ssim_pooled, without a workspace argument.  The scratch
 * ssim_pooled would take from `ws` comes from one static device buffer of
 * ssimx_noalloc_scratch_bytes() bytes (8 MiB) per GPU, held from the first
 * call on that GPU until the process ends; a call whose ssimx_workspace_size
 * (SSIMX_OP_POOLED) exceeds it returns SSIMX_ESCRATCH before any launch.  The
 * call allocates no memory of any kind.  It runs on the calling thread's
 * current device, and `stream` must belong to that device.  Every call on a
 * GPU shares that GPU's buffer: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller. */
ssimx_status ssim_pooled_noalloc(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis, int batch,
                                 float* score_out, void* stream);
size_t ssimx_noalloc_scratch_bytes(void);

/* MS-SSIM over n_scales (1..8) dyadic scales built by 2x2 averaging (odd
 * sizes floored).  weights: HOST float [n_scales] exponents.
 * score_out: float32 [batch] = S_M^{w_M} prod_{j<M} CS_j^{w_j} (with
 * SSIMX_MS_SUM: w_M S_M + sum_{j<M} w_j CS_j, weights normalised).
 * cs_out (nullable): float32 [batch][n_scales]; entries 0..M-2 hold CS_j (mean
 * cs map), entry M-1 holds S_M (mean l*cs at the coarsest scale, or
 * mean(l) * mean(cs) with SSIMX_MS_COARSE_SEPARATE).
 * Every scale must hold at least one window (else ETOOSMALL). */
ssimx_status msssim(const ssimx_params* p, const float* weights, int n_scales, int flags,
                    const ssimx_image* ref, const ssimx_image* dis, int batch,
                    float* score_out, float* cs_out, void* ws, size_t ws_bytes, void* stream);

/* Host only.  Where msssim leaves its pyramid.  After an msssim call with the
 * same params, dtype, sizes, batch and n_scales returns, its workspace holds
 * the 2x2-average levels of scales j = 1 .. n_scales-1 (level j has
 * floor(H / 2^j) x floor(W / 2^j) pixels: MS-SSIM implementation list of the
 * "Versions of SSIM" section) of both planes as float32
 * [batch][heights[j]][widths[j]], dense, at byte offsets x_offsets[j] (ref)
 * and y_offsets[j] (dis) from the workspace base; for j = 0 (the caller's own
 * planes) the offsets are -1.  On integer planes every level is the exact
 * block mean (a multiple of 4^-j).  The four output arrays are HOST arrays of
 * n_scales entries; any may be NULL. */
ssimx_status ssimx_msssim_pyramid_layout(const ssimx_params* p, int dtype, int width, int height, int batch,
                                         int n_scales, int64_t* x_offsets, int64_t* y_offsets, int* widths,
                                         int* heights);

/* Adjoint of ssim_map with respect to dis:
 *   grad_dis(q) = sum_p grad_map(p) dQ(p)/d dis(q).
 * grad_map: float32 in the map layout (map_pitch, map_batch_stride).
 * grad_dis: float32 [batch][height][grad_pitch], frame stride
 * grad_batch_stride; fully overwritten.  Moments are recomputed, not stored. */
ssimx_status ssim_map_backward(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis,
                               int batch, const float* grad_map, int64_t map_pitch, int64_t map_batch_stride,
                               float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                               void* ws, size_t ws_bytes, void* stream);

/* Adjoint of ssim_pooled: grad_score float32 [batch] (dL/dscore). */
ssimx_status ssim_pooled_backward(const ssimx_params* p, const ssimx_image* ref, const ssimx_image* dis,
                                  int batch, const float* grad_score,
                                  float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                                  void* ws, size_t ws_bytes, void* stream);

/* Adjoint of msssim (same weights / flags): grad_score float32 [batch].
 * The pyramid and per-scale terms are recomputed. */
ssimx_status msssim_backward(const ssimx_params* p, const float* weights, int n_scales, int flags,
                             const ssimx_image* ref, const ssimx_image* dis, int batch,
                             const float* grad_score,
                             float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                             void* ws, size_t ws_bytes, void* stream);

/* The same adjoint for a caller that has already run msssim on these inputs
 * with these weights, n_scales and flags (a training loss): fwd_score float32
 * [batch] and fwd_cs float32 [batch][n_scales] are that call's score_out and
 * cs_out (device, read only).  The per-scale windowed passes of the forward
 * are not repeated; only the 2x2 pyramid is rebuilt, so the gradient is the
 * one msssim_backward gives.  Null fwd_score or fwd_cs: SSIMX_EINVAL.
 * SSIMX_MS_COARSE_SEPARATE returns SSIMX_ENOTSUP (its split coarsest term is
 * not in cs_out).  Workspace: the msssim_backward size. */
ssimx_status msssim_backward_values(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                    const ssimx_image* ref, const ssimx_image* dis, int batch,
                                    const float* fwd_score, const float* fwd_cs, const float* grad_score,
                                    float* grad_dis, int64_t grad_pitch, int64_t grad_batch_stride,
                                    void* ws, size_t ws_bytes, void* stream);

/* Exact integer window sums of a rectangular k x k window (Performance-
 * Efficiency subsection): sums_out int32 [5][batch][map_h][map_w] holding
 * S1x, S1y, S2x, S2y, S12 in that order (x = ref, y = dis), valid windows at
 * stride `stride`.  Integer dtypes only; every sum must fit in int32
 * (k^2 * maxval^2 < 2^31). */
ssimx_status ssimx_box_sums(int k, int stride, int algo, const ssimx_image* ref, const ssimx_image* dis,
                            int batch, int32_t* sums_out, void* ws, size_t ws_bytes, void* stream);

/* The five integral images of eq. integral_image_start and the four after it:
 * sat_out uint32 [5][batch][height+1][width+1] (zero first row and column,
 * entry (i,j) = sum over rows < i and cols < j of x, y, x^2, y^2, x*y,
 * modulo 2^32).  Integer dtypes only. */
ssimx_status ssimx_integral_images(const ssimx_image* ref, const ssimx_image* dis, int batch,
                                   uint32_t* sat_out, void* stream);

/* ---------------- spatial pooling of quality maps -------------------------
 * The pooling methods of the Spatial and Temporal Aggregation section,
 * applied per frame to a float32 map (e.g. the output of ssim_map).  With
 * n = w*h map positions and mu the map mean:
 *   MEAN             (1/n) sum Q
 *   COV              sigma_Q / mu, population sigma (the CoV equation)
 *   MEAN_DEV         (((1/n) sum |Q - mu|^p)^(1/p))^o      (p > 0)
 *   MINKOWSKI        (1/n) sum (1 - Q)^p                   (p > 0)
 *   DIST_WEIGHTED    sum (1-Q)^p Q / sum (1-Q)^p; 1 when every Q == 1 (p >= 0)
 *   FIVE_NUMBER      (min + Q1 + median + Q3 + max) / 5, quantiles by linear
 *                    interpolation between the order statistics at rank
 *                    floor((n-1) q) and the next one
 *   PERCENTILE       the m = ceil(p n / 100) smallest values divided by r,
 *                    then the mean                          (0 <= p <= 100, r > 0)
 * and, from the Moment-Based Pooling subsection and the windowed means after
 * the CoV equation (the paper uses them on the series of frame scores: pass
 * a batch of 1 x T maps, one row of T frame scores per video):
 *   GEOMETRIC        exp((1/n) sum log Q); 0 with a zero value, NaN with a
 *                    negative one
 *   HARMONIC         n / sum (1/Q); 0 with a zero value
 *   MEDIAN           the interpolated median (rank (n-1)/2)
 *   WIN_AM, WIN_GM,  mean over the n-p+1 windows of p consecutive values of
 *   WIN_HM, WIN_COV  the window's arithmetic / geometric / harmonic mean or
 *                    CoV; p an integer in 1..n (ETOOSMALL if p > n), the map
 *                    must be a single row (h == 1, else EINVAL)
 * Sums are accumulated in float64 in a fixed order (deterministic); order
 * statistics are exact (radix select on the float bit patterns). */
typedef enum {
  SSIMX_POOL_MEAN = 0,
  SSIMX_POOL_COV = 1,
  SSIMX_POOL_MEAN_DEV = 2,
  SSIMX_POOL_MINKOWSKI = 3,
  SSIMX_POOL_DIST_WEIGHTED = 4,
  SSIMX_POOL_FIVE_NUMBER = 5,
  SSIMX_POOL_PERCENTILE = 6,
  SSIMX_POOL_GEOMETRIC = 7,
  SSIMX_POOL_HARMONIC = 8,
  SSIMX_POOL_MEDIAN = 9,
  SSIMX_POOL_WIN_AM = 10,
  SSIMX_POOL_WIN_GM = 11,
  SSIMX_POOL_WIN_HM = 12,
  SSIMX_POOL_WIN_COV = 13
} ssimx_pool_kind;

typedef struct {
  int kind; /* ssimx_pool_kind */
  double p;  /* order / exponent / percentile, per kind */
  double o;  /* outer exponent of MEAN_DEV */
  double r;  /* divisor of PERCENTILE */
} ssimx_pool;

/* Workspace bytes of ssimx_pool_map (host only). */
ssimx_status ssimx_pool_workspace_size(const ssimx_pool* pool, int w, int h, int batch, size_t* bytes);

/* map: float32 device, element (b, i, j) at b*batch_stride + i*pitch + j;
 * out: float32 device [batch].  Host validation: EINVAL for a bad kind or
 * parameter, null pointers, pitch < w; ETOOSMALL for an empty map; ENOTSUP for
 * maps of 2^31 positions or more; EWORKSPACE for a missing or short workspace.
 * Asynchronous on `stream`. */
ssimx_status ssimx_pool_map(const ssimx_pool* pool, const float* map, int w, int h, long long pitch,
                            long long batch_stride, int batch, float* out, void* ws, size_t ws_bytes, void* stream);

/* Pre-scaled, pooled SSIM (Transforming-across-Scales subsection and the
 * aggregation section): both planes are down-sampled by f x f block averages
 * (f = factor; 0 selects the subsection's max(1, ceil(height / 256)); 1 keeps
 * the planes), the SSIM map with params p is formed on the float32 result,
 * and each frame's map is pooled by `pool`.  score_out: float32 device
 * [batch].  The paper's "Enhanced SSIM" composition is p = {BOX, k 11,
 * stride 5}, factor 0, pool COV.  The integral-image method needs integer
 * planes, so it is ENOTSUP with a factor other than 1.  Workspace: size from
 * ssimx_scaled_pooled_workspace_size. */
ssimx_status ssimx_scaled_pooled_workspace_size(const ssimx_params* p, int factor, const ssimx_pool* pool, int dtype,
                                                int w, int h, int batch, size_t* bytes);
ssimx_status ssimx_scaled_pooled_ssim(const ssimx_params* p, int factor, const ssimx_pool* pool,
                                      const ssimx_image* ref, const ssimx_image* dis, int batch, float* score_out,
                                      void* ws, size_t ws_bytes, void* stream);

/* Channel-wise colour SSIM (Channel-wise SSIM subsection): YCbCr by the BT.709
 * transform printed there (Y = 0.213 R + 0.715 G + 0.072 B, Cb = 0.539 (B - Y),
 * Cr = 0.635 (R - Y)), the pooled SSIM of each channel with params p (the same
 * window and C1, C2 for all three), and
 *   score = (SSIM_Y + alpha SSIM_Cb + beta SSIM_Cr) / (1 + alpha + beta);
 * alpha = beta = 0.125 is the 0.8 / 0.1 / 0.1 weighting of FFMPEG and Daala.
 * rgb: planar u8/u16/f32/bf16, element (b, c, r, col) at b*batch_stride +
 * c*channel_stride + r*pitch + col.  score_out float32 [batch];
 * channel_scores nullable float32 [batch][3].  EINVAL when 1 + alpha + beta
 * is 0; ENOTSUP for the integral-image algorithm (channel planes are float32).
 * Workspace: ssimx_color_workspace_size. */
ssimx_status ssimx_color_workspace_size(const ssimx_params* p, int w, int h, int batch, size_t* bytes);
ssimx_status ssimx_color_ssim(const ssimx_params* p, double alpha, double beta, const void* ref_rgb,
                              const void* dis_rgb, int dtype, int w, int h, int64_t pitch, int64_t channel_stride,
                              int64_t batch_stride, int batch, float* score_out, float* channel_scores, void* ws,
                              size_t ws_bytes, void* stream);

/* ---------------- SSIM-3D / MS-SSIM-3D ------------------------------------
 * Spatio-Temporal SSIM subsection: SSIM whose mean, variance and covariance
 * are taken over k x k x kt rectangular spatio-temporal boxes (equal weights,
 * N = k^2 kt samples).  Map frame t, position (i, j) covers frames t..t+kt-1,
 * rows i..i+k-1 and columns j..j+k-1 of the clip; boxes lie inside the clip in
 * every axis, so a clip of `frames` frames gives frames-kt+1 map frames of
 * (height-k+1) x (width-k+1).  Computed with rolling temporal sums (add the
 * entering frame, drop the leaving one), so the cost per frame is independent
 * of kt.
 *
 * p: window must be SSIMX_WIN_BOX, stride 1, SSIMX_PAD_VALID, k <= 16
 *    (else ENOTSUP); algo is ignored.  kt: 1..64 (else EINVAL).
 * ref, dis: clips of `frames` frames; frame f of a clip is its image `f`
 *    (batch_stride apart), row pitch at most 2^26 elements (else EINVAL).
 *    Any dtype: 8-bit clips use exact uint32 sums, others float64 sums.
 * map_out (nullable): float32 [frames-kt+1][height-k+1][map_pitch] with frame
 *    stride map_frame_stride; score_out (nullable, not both null): float32
 *    [frames-kt+1] mean of each map frame.
 * frames < kt or a frame smaller than the window: ETOOSMALL.
 * Workspace: ssimx_ssim3d_workspace_size. */
ssimx_status ssimx_ssim3d_workspace_size(const ssimx_params* p, int kt, int dtype, int width, int height, int frames,
                                         size_t* bytes);
ssimx_status ssimx_ssim3d(const ssimx_params* p, int kt, const ssimx_image* ref, const ssimx_image* dis, int frames,
                          float* map_out, long long map_pitch, long long map_frame_stride, float* score_out,
                          void* ws, size_t ws_bytes, void* stream);

/* MS-SSIM-3D: every frame of both clips is reduced by the 2x2-average pyramid
 * of msssim (the temporal extent is unchanged); at each scale the SSIM-3D map
 * frames give CS_j(t) (mean cs, j < M) and S_M(t) (mean l*cs at the coarsest
 * scale), combined per map frame t exactly as msssim combines them (weights
 * and flags as for msssim, SSIMX_MS_SUM included).  Every scale must hold at
 * least one window.  score_out: float32 [frames-kt+1]; cs_out (nullable):
 * float32 [frames-kt+1][n_scales] in the layout of msssim.
 * Workspace: ssimx_msssim3d_workspace_size. */
ssimx_status ssimx_msssim3d_workspace_size(const ssimx_params* p, int kt, int n_scales, int dtype, int width,
                                           int height, int frames, size_t* bytes);
ssimx_status ssimx_msssim3d(const ssimx_params* p, int kt, const float* weights, int n_scales, int flags,
                            const ssimx_image* ref, const ssimx_image* dis, int frames, float* score_out,
                            float* cs_out, void* ws, size_t ws_bytes, void* stream);

/* Colour front end of the differentiable-loss workload: BT.601 luma
 * Y = 0.299 R + 0.587 G + 0.114 B of planar RGB (the paper's Channel-wise SSIM
 * subsection prints the BT.709 matrix; BT.601 weights are used here).
 * rgb: float32 or bfloat16 planes, element (b, c, r, col) at
 * b*batch_stride + c*channel_stride + r*pitch + col.
 * y_out: float32 [batch][height][width], contiguous. */
ssimx_status ssimx_rgb_to_luma(const void* rgb, int dtype, int width, int height, int64_t pitch,
                               int64_t channel_stride, int64_t batch_stride, int batch, float* y_out, void* stream);
/* Adjoint: grad_rgb(b, c, r, col) = weight_c * grad_y(b, r, col) (overwrites).
 * grad_y: float32 [batch][height][width] contiguous; grad_rgb: float32 with
 * the given strides. */
ssimx_status ssimx_luma_grad_to_rgb(const float* grad_y, int width, int height, int batch, float* grad_rgb,
                                    int64_t pitch, int64_t channel_stride, int64_t batch_stride, void* stream);

/* ---------------- ragged batches ------------------------------------------
 * A plan covers n independent pairs, each with its own size and params.  It
 * owns a device descriptor table, a partial-sum buffer and an instantiated
 * hipGraph of one persistent launch plus a per-pair finalise.  Pair buffers
 * must stay valid (same addresses) for the plan's lifetime. */
typedef struct {
  ssimx_image ref, dis;  /* single frame each */
  ssimx_params p;
  float* map_out;        /* nullable: map of this pair */
  int64_t map_pitch;
} ssimx_pair;

typedef struct ssimx_plan ssimx_plan;

/* pairs: HOST array [n].  tile shapes come from the autotune cache when an
 * entry exists (see ssimx_autotune), else from built-in defaults. */
ssimx_status ssimx_plan_create(const ssimx_pair* pairs, int n, void* stream, ssimx_plan** out);
/* scores_out: float32 [n] device; one graph launch on `stream`. */
ssimx_status ssimx_plan_run(ssimx_plan* plan, float* scores_out, void* stream);
/* Same work as ssimx_plan_run, but one ordinary launch sequence per pair
 * (the unbatched baseline). */
ssimx_status ssimx_plan_run_unbatched(ssimx_plan* plan, float* scores_out, void* stream);
ssimx_status ssimx_plan_destroy(ssimx_plan* plan);
/* Host: number of (pair, tile) work items and persistent blocks of a plan. */
ssimx_status ssimx_plan_info(const ssimx_plan* plan, int* n_items, int* n_blocks);

/* ---------------- differentiable MS-SSIM loss (training objective) ---------
 * The use of MS-SSIM as a training objective (Off-the-shelf Performance
 * subsection) in one call: BT.601 luma Y = 0.299 R + 0.587 G + 0.114 B of two
 * planar RGB batches (dtype SSIMX_F32 or SSIMX_BF16; element (b, c, r, x) at
 * b * batch_stride + c * channel_stride + r * pitch + x, strides in elements),
 * MS-SSIM of the luma planes with msssim's weights / n_scales / flags
 * semantics, and
 *   loss_out[0] = (1 / batch) sum_b (1 - MS-SSIM_b)      (device float [1]),
 * score_out (nullable, device float [batch]) the per-frame MS-SSIM, and
 * grad_rgb (nullable) d loss / d dis_rgb in grad_dtype (SSIMX_F32 or
 * SSIMX_BF16, rounded to nearest even), same layout rules with grad_pitch,
 * grad_channel_stride, grad_batch_stride.  The gradient is msssim_backward's
 * adjoint (moments recomputed) through the luma map; nothing is kept between
 * calls.  Workspace: ssimx_msssim_loss_workspace_size (any grad_dtype). */
ssimx_status ssimx_msssim_loss_workspace_size(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                              int dtype, int width, int height, int batch, size_t* bytes);
ssimx_status ssimx_msssim_loss_rgb(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                   const void* ref_rgb, const void* dis_rgb, int dtype, int width, int height,
                                   int64_t pitch, int64_t channel_stride, int64_t batch_stride, int batch,
                                   float* loss_out, float* score_out, void* grad_rgb, int grad_dtype,
                                   int64_t grad_pitch, int64_t grad_channel_stride, int64_t grad_batch_stride,
                                   void* ws, size_t ws_bytes, void* stream);

/* The same evaluation in two calls, for autograd-style callers whose upstream
 * d(objective)/d(loss) is known only later.  _deferred computes loss_out and
 * score_out as ssimx_msssim_loss_rgb does and leaves the luma-level gradients
 * of the loss in ws; _grad (same p, weights, n_scales, flags, dtype, sizes and
 * ws, any later point on the stream, ws untouched in between) writes
 * grad_rgb = upstream[0] * d loss / d dis_rgb, upstream a device float [1]
 * (nullable: 1).  With upstream null or 1 the gradient equals
 * ssimx_msssim_loss_rgb's bit for bit. */
ssimx_status ssimx_msssim_loss_rgb_deferred(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                            const void* ref_rgb, const void* dis_rgb, int dtype, int width,
                                            int height, int64_t pitch, int64_t channel_stride, int64_t batch_stride,
                                            int batch, float* loss_out, float* score_out, void* ws, size_t ws_bytes,
                                            void* stream);
ssimx_status ssimx_msssim_loss_rgb_grad(const ssimx_params* p, const float* weights, int n_scales, int flags,
                                        int dtype, int width, int height, int batch, const float* upstream,
                                        void* grad_rgb, int grad_dtype, int64_t grad_pitch,
                                        int64_t grad_channel_stride, int64_t grad_batch_stride, const void* ws,
                                        size_t ws_bytes, void* stream);

/* A loss plan: the same computation for one shape, replayed as one HIP graph.
 * Create allocates the plan's workspace and a device argument block (and a
 * small pinned ring); the first run with and the first run without a
 * gradient each capture the launches once.  Every run copies its pointers
 * and strides into the argument block (one asynchronous host-to-device copy on
 * `stream`, ordered before the graph), so new tensors need no new capture.
 * Results equal ssimx_msssim_loss_rgb's bit for bit.  Runs of one plan must be
 * issued on one stream (or otherwise serialised): they share the plan's
 * workspace and argument block.  Destroy after the last run has completed. */
typedef struct ssimx_loss_plan ssimx_loss_plan;
ssimx_status ssimx_loss_plan_create(const ssimx_params* p, const float* weights, int n_scales, int flags, int dtype,
                                    int grad_dtype, int width, int height, int batch, ssimx_loss_plan** out);
ssimx_status ssimx_loss_plan_run(ssimx_loss_plan* plan, const void* ref_rgb, const void* dis_rgb, int64_t pitch,
                                 int64_t channel_stride, int64_t batch_stride, float* loss_out, float* score_out,
                                 void* grad_rgb, int64_t grad_pitch, int64_t grad_channel_stride,
                                 int64_t grad_batch_stride, void* stream);
ssimx_status ssimx_loss_plan_destroy(ssimx_loss_plan* plan);

/* ---------------- autotuning ----------------------------------------------
 * Times the candidate tile shapes of the forward kernel for (params, dtype,
 * width, height, batch) on `stream` (allocating and freeing its own scratch
 * frames) and records the fastest in the process-wide cache.  The cache is
 * read by every later call and plan.  Mutex-guarded. */
ssimx_status ssimx_autotune(const ssimx_params* p, int dtype, int width, int height, int batch, void* stream,
                            int* best_tile_out);
/* Load / save the cache as JSON (path: host string):
 *   {"version": SSIMX_VERSION, "entries": {"<key>": <tile index>, ...}}
 * Load is strict and all-or-nothing: a missing file, a file of 1 MiB or more,
 * another version, a tile index outside 0..ssimx_num_tile_configs()-1, a
 * duplicate key, a key with a quote, backslash or non-printable byte or over
 * 191 bytes, or anything else malformed returns SSIMX_EINVAL and leaves the
 * cache unchanged; otherwise the entries are merged into the cache.
 * Environment: SSIMX_TUNE_CACHE=<path> loads that file once, before the
 * process's first tile choice, autotune or save call (a missing or malformed
 * file loads nothing), and ssimx_autotune
 * writes the whole cache back to it. */
ssimx_status ssimx_tune_cache_load(const char* path);
ssimx_status ssimx_tune_cache_save(const char* path);
/* Force a tile configuration index for later calls (-1 = automatic). */
ssimx_status ssimx_set_tile_override(int tile);
/* Number of tile configurations known to the forward kernel. */
int ssimx_num_tile_configs(void);

const char* ssimx_strerror(int status);
int ssimx_last_hip_error(void);
int ssimx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SSIMX_H */
