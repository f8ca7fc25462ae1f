/*
 * hb.h - C ABI of the MI355X (gfx950) haemoglobin-estimation library.
 *
 * Implements the per-frame path of Jones et al., "Fast Estimation of
 * Haemoglobin Concentration in Tissue Via Wavelet Decomposition"
 * (arXiv 1706.07263), Method section:
 *   1. RGB log-attenuation y = -ln(max(I, floor));
 *   2. n-level 2D Haar transform of each channel (Eq. 1-2, 2x2 windows);
 *   3. Tikhonov inversion of every directional coefficient to (Hb, HbO2)
 *      with M = (E'E + gamma I)^-1 E' (Eq. 5 with the camera matrix replaced
 *      by E, the Jacobian of the RGB forward model at a reference point);
 *   4. on the low-pass band, the posterior mean of (Hb, HbO2) over a
 *      THb x SO2 grid, Gaussian likelihood on the block-mean log-attenuation
 *      through the nonlinear forward model, uniform prior over the nodes
 *      (the paper applies a Bayesian estimator to this band; the low-pass
 *      coefficients behave as a lower-resolution image);
 *   5. inverse Haar (Eq. 4: H is its own inverse) to full-resolution Hb, HbO2,
 *      and the derived maps THb = Hb + HbO2, SO2 = HbO2 / THb (Fig. 1).
 *
 * Conventions
 *   - Every function returns hb_status_t; no exception or abort crosses the ABI.
 *   - Argument, shape and state errors are detected on the host before any
 *     device work; nothing is launched when a call fails.
 *   - Device pointers are plain HIP device addresses (e.g. a PyTorch tensor's
 *     data_ptr()); the caller owns frames and output maps.  The plan owns its
 *     tables and scratch, all allocated in hb_plan_create/hb_set_forward_model.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - A plan is bound to one device and is not re-entrant: calls that use the
 *     same plan on different streams must be ordered by the caller.
 */
#ifndef HB_H
#define HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HB_OK = 0,
    HB_ERR_INVALID_ARG = -1,      /* NULL pointer, value out of range            */
    HB_ERR_SHAPE = -2,            /* frame size not divisible by 2^levels, ...   */
    HB_ERR_NO_FORWARD_MODEL = -3, /* hb_estimate_frames before the model is set  */
    HB_ERR_OUT_OF_MEMORY = -4,    /* device allocation failed                    */
    HB_ERR_DEVICE = -5,           /* a HIP call or kernel launch failed          */
    HB_ERR_ILL_POSED = -6,        /* E'E + gamma I is singular                   */
    HB_ERR_BATCH = -7,            /* n_frames > max_batch                        */
    HB_ERR_SCRATCH = -8           /* hb_estimate_frames_noalloc: the call's
                                     buffers exceed HB_NOALLOC_SCRATCH_BYTES     */
} hb_status_t;

/* Size of the static per-device scratch array of hb_estimate_frames_noalloc. */
#define HB_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

typedef enum { HB_F32 = 0, HB_F16 = 1, HB_BF16 = 2 } hb_dtype_t;

/* Estimator on the low-pass band.  TIKHONOV applies the linearised inverse there
 * too (the paper notes Tikhonov can be used on any Haar coefficient); it is a
 * diagnostic mode: the whole path then reduces to one affine map per pixel. */
typedef enum { HB_LOWPASS_BAYES = 0, HB_LOWPASS_TIKHONOV = 1 } hb_lowpass_t;

typedef struct hb_plan_s *hb_plan_t;

/* Plan descriptor.  Fill with hb_plan_desc_default, then override. */
typedef struct {
    int32_t width, height;      /* frame size in pixels; both divisible by 2^levels      */
    int32_t levels;             /* Haar levels n, 0..5 (0 = posterior on every pixel)    */
    int32_t frame_dtype;        /* hb_dtype_t of the stored intensities                   */
    int32_t max_batch;          /* largest n_frames per hb_estimate_frames call (>= 1)   */
    int32_t grid_thb, grid_so2; /* posterior grid nodes along THb and SO2 (1..4096 each) */
    double thb_min, thb_max;    /* uM, inclusive linspace                                  */
    double so2_min, so2_max;    /* fraction in [0, 1], inclusive linspace                  */
    double lambda;              /* Tikhonov gamma relative to tr(E'E)/2 (>= 0)             */
    double sigma;               /* likelihood s.d. in natural-log attenuation units (> 0) */
    double intensity_floor;     /* intensities below it are clamped before the log (> 0) */
    double ref_thb, ref_so2;    /* linearisation point of E; NaN = grid centre            */
    double thb_eps;             /* SO2 is NaN where THb <= thb_eps (uM)                    */
    int32_t lowpass;            /* hb_lowpass_t                                            */
    int32_t grid_split;         /* posterior grid split across workgroups; 0 = automatic
                                   (sized so that max_batch frames fill the GPU)         */
    int32_t illumination;       /* 1: the low-pass posterior integrates out an unknown
                                   per-pixel log offset b*(1,1,1) under a flat prior
                                   (the constant attenuation term for global illumination,
                                   Method, before Eq. 9): residuals are projected onto the
                                   plane orthogonal to (1,1,1).  0 (default) = off.  Only
                                   affects HB_LOWPASS_BAYES; any other value is rejected. */
    double posterior_tolerance; /* uM, finite.  > 0: the posterior skips 4x4-node grid chunks
                                   whose weights are all provably below 2^-T of the pixel's
                                   reference weight and, up to a per-wave budget of B
                                   chunks, chunks below 2^-(T-6), with T and B chosen so
                                   that the skipped weights move the posterior mean of Hb
                                   and HbO2 by at most this much (bound: 2 thb_max (G 2^-T
                                   + 16 B S 2^-(T-6)), G grid nodes, S grid splits;
                                   T = ceil(log2(2 G thb_max / tolerance)) + 1; T, B and
                                   the bound are reported by hb_plan_get_info).
                                   0: skip only chunks whose float32 weights are all exactly
                                   zero (T = 160; results equal those of no skipping, bit
                                   for bit).  < 0: skip nothing (every chunk that holds a
                                   grid node is evaluated; T = +inf).  Default 1e-6 uM, 1%
                                   of the FP32 parity tolerance.                          */
} hb_plan_desc_t;

/* Camera sensitivities and attenuation spectra (the camera matrix C and the
 * coefficients xi of the Method section).  Copied by hb_set_forward_model. */
typedef struct {
    int32_t n_wavelengths;
    const double *wavelength_nm;  /* [n], informational, may be NULL               */
    const double *eps_hb;         /* [n] cm^-1 uM^-1, natural-log units             */
    const double *eps_hbo2;       /* [n]                                            */
    const double *response;       /* [3][n] R, G, B; each row normalised to unit sum */
    double path_length_cm;        /* > 0                                             */
} hb_forward_model_t;

/* Output maps, device pointers, each [n_frames][height][width] float32,
 * planar.  Any pointer may be NULL to skip that map. */
typedef struct {
    float *hb, *hbo2, *thb, *so2;
} hb_maps_t;

/* Plan-time quantities, for inspection and tests. */
typedef struct {
    double E[6];          /* 3x2 row-major Jacobian at the reference point (built on the device, FP64) */
    double M[6];          /* 2x3 row-major Tikhonov operator (Hb row, HbO2 row), FP64                  */
    double gamma;         /* absolute gamma = lambda * tr(E'E) / 2                                     */
    double ref_hb, ref_hbo2;
    double mu_ref[3];     /* centring offset: -ln of the float32 reference intensities                 */
    int32_t grid_split;   /* posterior grid split in use                                                */
    int32_t n_tiles;      /* grid super-tiles                                                           */
    int32_t posterior_kernel; /* 0 = MFMA logits, 1 = direct VALU (grids too coarse for the former),
                                 2 = direct VALU with double-float logits (grids whose neighbouring nodes
                                 are too far apart for float32 logits: direct_index > 3800)             */
    int64_t n_nodes;
    double skip_log2;     /* T: chunks whose logit bound lies more than T below the reference are skipped
                             (+inf: nothing is skipped)                                                   */
    double skip_bound;    /* uM, the stated bound on the posterior-mean change from skipping (0: exact)  */
    double mfma_index;    /* R^2 h: squared super-tile radius (scaled log-attenuation units) times the
                             node spacing (uM).  The MFMA kernel runs when it is <= 700 (for pixels
                             far from the nodes see far_room)                                          */
    double direct_index;  /* max over neighbouring grid nodes of their squared scaled distance times their
                             largest Hb/HbO2 difference (uM); float32 logits can move a posterior mean by
                             about 8e-9 times this                                                        */
    double band_log2;     /* chunks whose logit bound lies between band_log2 and skip_log2 below the
                             reference are skipped too, up to band_chunks of them per wave (a wave
                             covers 32 or 64 pixels); band_log2 = skip_log2: no such budget            */
    int64_t band_chunks;
    double far_room;      /* how far (scaled units) an observation may lie from the grid's nodes
                             before the posterior kernel's float32 logits exceed its precision budget;
                             the kernel forms the sums of pixels lying farther than this (soft minimum
                             over the nodes) again with double-float logits (hb_plan_get_far_pixels).
                             MFMA kernel: max(3, 350 / (R h) - R), its expanded logit's terms growing
                             as (R + distance) R; float32 direct kernel: sqrt(1000 / h), its
                             differences rounding at the scale of the distance; +inf for the direct
                             kernel with double-float logits                                           */
    int32_t mfma_df_constant; /* 1: the MFMA kernel sums its pixel operand's constant |r|^2 + m as a
                             double-float (mfma_index > 350)                                           */
    double m_norm;        /* |M|inf, uM per unit log-attenuation                                         */
    int32_t k1_double_float; /* 1: the log + Haar kernel forms log-ratios, Haar coefficients and the
                             Tikhonov apply as double-floats (|M|inf > 1100 or three or more levels:
                             float32 log-ratios would reach the maps at up to ~1e-4 uM)               */
} hb_plan_info_t;

/* Fill `desc` with defaults: 64x64, 1 level, FP32, max_batch 1, grid 128x128
 * over THb [20,200] uM x SO2 [0.3,1], lambda 1e-3, sigma 0.01, floor 1e-4,
 * reference = grid centre, thb_eps 1e-3, Bayesian low-pass, automatic split. */
hb_status_t hb_plan_desc_default(hb_plan_desc_t *desc);

/* Validate `desc` and allocate the plan on `device` (hipMalloc happens here
 * and in hb_set_forward_model only).  On failure *out is set to NULL. */
hb_status_t hb_plan_create(const hb_plan_desc_t *desc, int device, hb_plan_t *out);

/* Set the forward model: builds E and M on the device (FP64, the only double-
 * precision device code), the centred posterior grid table on the host (FP64
 * rounded to FP32), and uploads it.  Synchronous.  HB_ERR_ILL_POSED if
 * E'E + gamma I is singular.  May be called again to replace the model. */
hb_status_t hb_set_forward_model(hb_plan_t plan, const hb_forward_model_t *fm);

/* Estimate n_frames frames.  d_frames: device, [n][height][width][3] of the
 * plan's dtype (HWC interleaved R,G,B).  d_out: host struct of device map
 * pointers.  Asynchronous on `stream`; it neither allocates nor synchronises,
 * so it may be captured into a HIP graph.  n_frames == 0 is a no-op. */
hb_status_t hb_estimate_frames(hb_plan_t plan, const void *d_frames, int32_t n_frames,
                               const hb_maps_t *d_out, void *stream);

/* hb_estimate_frames for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bit for bit, but the call's
 * intermediate buffers live in a static device array of
 * HB_NOALLOC_SCRATCH_BYTES that the library holds on each device until the
 * process ends (set up by hb_plan_create), instead of the plan's own scratch.
 * The call allocates and frees nothing.  Arguments, ownership and errors are
 * those of hb_estimate_frames, plus HB_ERR_SCRATCH (nothing launched) when
 * n_frames frames need more than the array: per frame, 24 B per low-pass
 * pixel (observation) + 8 B per pixel (detail part) + 24 B x grid_split per
 * low-pass pixel (posterior partials, Bayesian low-pass only) + 4 B per
 * low-pass pixel (split grids only) + 8 B per low-pass pixel (estimate), each
 * buffer rounded up to 256 B (one 1920x1080 frame at 2 levels and one split:
 * 23.8 MB; one 3840x2160 frame at 2 levels: 95 MB).  Every call on a device
 * shares that device's array and leaves its contents there: calls of this
 * function that overlap in time on one device (different streams, plans or
 * host threads) race and give wrong results; calls ordered on one stream do
 * not.  hb_debug_copy shows the buffers of hb_estimate_frames calls only. */
hb_status_t hb_estimate_frames_noalloc(hb_plan_t plan, const void *d_frames, int32_t n_frames,
                                       const hb_maps_t *d_out, void *stream);

/* Wait for the plan's last hb_estimate_frames call (not for other streams, and
 * not for replays of graphs the caller captured: those are the caller's to wait
 * for), then free the plan's device memory.  NULL is accepted. */
hb_status_t hb_destroy(hb_plan_t plan);

/* Static description of a status code (never NULL). */
const char *hb_status_string(hb_status_t status);

/* Device bytes the plan holds (tables + scratch for max_batch), 0 for NULL. */
size_t hb_plan_device_bytes(hb_plan_t plan);

/* Copy out the plan-time quantities.  HB_ERR_NO_FORWARD_MODEL before the
 * model is set. */
hb_status_t hb_plan_get_info(hb_plan_t plan, hb_plan_info_t *info);

/* Per-kernel timing: when enabled, hb_estimate_frames records HIP events
 * around each of its kernels on its stream (up to 4096 calls are kept).
 * hb_plan_get_timing waits for the recorded events, returns the summed
 * milliseconds and launch counts of the four stages
 *   [0] log + Haar + Tikhonov, [1] posterior, [2] recomposition + maps,
 *   [3] whole call,
 * and clears the record. */
hb_status_t hb_plan_set_timing(hb_plan_t plan, int32_t enable);
hb_status_t hb_plan_get_timing(hb_plan_t plan, double ms[4], int64_t launches[4]);

/* Posterior work of the calls made since the last hb_plan_set_timing
 * (counted only while timing is enabled): `evaluated` = (LL pixel, grid node)
 * pairs the posterior kernel actually evaluated (whole 16-node chunks for
 * every pixel of a wave), `full` = LL pixels x grid nodes of those calls.
 * The kernels leave out chunks whose weights lie more than T below every
 * pixel's reference weight (posterior_tolerance above), so evaluated <= full;
 * the results then move by at most the plan's stated skip_bound (exactly 0
 * for T = 160 and for no skipping).  Synchronises the device. */
hb_status_t hb_plan_get_work(hb_plan_t plan, int64_t *evaluated, int64_t *full);

/* Posterior sums of the calls made since the last hb_plan_set_timing
 * (counted only while timing is enabled) that the posterior kernel formed again
 * with double-float logits, one per LL pixel and grid split (grid_split in
 * hb_plan_info_t): those of pixels whose observation lies farther than the
 * plan's far_room from the split's nodes (soft minimum of the scaled
 * distances, -log2 of the sum of 2^-d^2 over the nodes) and, with a split
 * grid, from the best probe node of the whole grid (the expanded logit
 * would round at the scale of that distance; the posterior of step 4 is
 * unchanged, only its precision).  Their pairs are not counted by
 * hb_plan_get_work.  Synchronises the device, then writes the count to the
 * host pointer `pixels`; HB_ERR_INVALID_ARG for a NULL plan or pointer,
 * HB_ERR_DEVICE if the device cannot be read. */
hb_status_t hb_plan_get_far_pixels(hb_plan_t plan, int64_t *pixels);

/* Intermediate buffers of the last hb_estimate_frames call, and the plan's
 * posterior operand tables, for step-by-step checks.  Synchronises the
 * device, then copies `bytes` from the start of the selected buffer of frame
 * `frame` into host memory (the tables ignore `frame`, which must still lie
 * in [0, max_batch); they need a forward model, else
 * HB_ERR_NO_FORWARD_MODEL):
 *   HB_DEBUG_LOWPASS_OBS: float32 [2][3][LL], centred low-pass observation
 *       z_k = ybar_k - mu_ref_k (ybar = block mean of log-attenuation) as a
 *       double-float: z_k = [0][k] + [1][k] (high and low parts),
 *       LL = (height >> levels) * (width >> levels), row-major blocks;
 *   HB_DEBUG_DETAILS: float32 [height][width][2], detail part of the maps
 *       (Hb, HbO2): the inverse Haar (Eq. 4) of the Tikhonov-inverted
 *       directional coefficients with the low-pass coefficient set to 0; the
 *       maps are this plus the block's low-pass estimate;
 *   HB_DEBUG_LOWPASS_EST: float32 [LL][2], low-pass estimate (Hb, HbO2)
 *       per block (the block mean of the output maps);
 *   HB_DEBUG_NODE_OPERANDS: float32 [n_chunks][4][16], per 16-node chunk of
 *       the posterior grid (n_chunks = grid nodes rounded up to whole
 *       super-tiles / 16) the scaled, centred node coordinates 0..2
 *       relative to their super-tile's centre, and minus their squared norm,
 *       as [coordinate or norm][node];
 *   HB_DEBUG_SPLIT_OPERANDS: bf16 bits (uint16) [n_chunks][4][16][8], the
 *       MFMA node operands built from those values: for row g < 3 and
 *       value v of node i, three bf16 parts with v1 + v2 + v3 = v exactly,
 *       stored as (v1, v2, v1, v3, v2, v1, v3, v2); for g = 3 the norm's
 *       parts and three ones, (n1, n2, n3, 1, 1, 1, 0, 0). */
typedef enum {
    HB_DEBUG_LOWPASS_OBS = 0,
    HB_DEBUG_DETAILS = 1,
    HB_DEBUG_LOWPASS_EST = 2,
    HB_DEBUG_NODE_OPERANDS = 3,
    HB_DEBUG_SPLIT_OPERANDS = 4
} hb_debug_buffer_t;
hb_status_t hb_debug_copy(hb_plan_t plan, int32_t which, int32_t frame, void *host_dst, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* HB_H */
