/*
 * asp.h -- C ABI of the MI355X (gfx950) Asp-Clean2016 minor cycle.
 *
 * Method: L. Zhang, S. Bhatnagar, U. Rau, M. Zhang (2016), "Efficient
 * implementation of the adaptive scale pixel decomposition algorithm".
 * One minor-cycle iteration (the loop of Sect. 2, steps 1-4, with the fit of
 * Sect. 3):
 *   1. find the peak of |residual|                  (Sect. 2 step 1; Sect. 3,
 *                                                      simple initial values)
 *   2. stop on a threshold or an iteration count    (Sect. 2 step 4)
 *   3. fit the active set of Gaussian components to the residual by
 *      Levenberg-Marquardt; with the PSF taken as one Gaussian, each
 *      component convolved with the PSF is an analytic Gaussian, so the
 *      objective needs no convolution                (Sect. 3, Eq. 4)
 *   4. scale the new component by the loop gain and subtract the fitted
 *      Gaussians from the residual                   (Sect. 3; Sect. 2 step 3)
 *   5. components are reported in the sky plane by analytic deconvolution of
 *      the Gaussian beam                             (Sect. 3, Eqs. 5-6)
 *
 * Conventions
 *   Images are FP32, row-major, H rows by W columns; pixel (r, c) is element
 *   r*W + c; its centre is at x = c, y = r.  H*W must be below 2^32 - 1.
 *   A Gaussian (a, x, y, s) is a * exp(-((c-x)^2 + (r-y)^2) / (2 s^2)),
 *   point-sampled at pixel centres; s is the standard deviation.  "Convolved"
 *   parameters are those of the fitted Gaussian (PSF (*) component); "sky"
 *   parameters are the component's own (Eqs. 5-6).
 * Ownership
 *   The context owns all device memory it allocates.  Host arrays passed in
 *   are copied and stay the caller's.  Device pointers passed to *_device
 *   calls must stay valid only for the duration of the call.  Outputs go to
 *   caller-provided buffers.
 * Errors
 *   Every call returns asp_status: negative values are errors (the context
 *   keeps a message, see asp_last_error), positive values report a stop.
 *   No C++ exception crosses this boundary.  A context is bound to one HIP
 *   stream and is not thread-safe; distinct contexts are independent.
 */
#ifndef ASP_H
#define ASP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASP_MAX_ACTIVE 16

typedef struct asp_ctx asp_ctx;

typedef enum {
    ASP_OK = 0,
    ASP_STOP_THRESHOLD = 1,      /* |peak| below the threshold (Sect. 2 step 4)  */
    ASP_STOP_MAXITER = 2,        /* iteration count reached (Sect. 2 step 4)     */
    ASP_LM_NOT_CONVERGED = 3,    /* the fit used its whole trial budget          */
    ASP_ERR_INVALID_ARG = -1,
    ASP_ERR_NONFINITE = -2,      /* NaN or Inf in an input image                 */
    ASP_ERR_PSF = -3,            /* PSF peak not positive                        */
    ASP_ERR_STATE = -4,          /* call out of order                            */
    ASP_ERR_CAPACITY = -5,       /* component list or output buffer full         */
    ASP_ERR_DEVICE = -6,         /* a HIP call failed                            */
    ASP_ERR_NOMEM = -7
} asp_status;

/* A Gaussian in convolved (fit) space. */
typedef struct { double amp, x, y, width; } asp_gauss;

/* One component.  flux = 2 pi amp width^2 (sky plane); amp/width are alpha_i
 * and omega_i of Eqs. 5-6; amp_c/width_c the fitted (convolved) amplitude
 * and width after the loop gain; is_point = 1 when omega_i <= 1e-6 omega_b,
 * then amp = 0 and flux carries the component. */
typedef struct {
    double flux, amp, x, y, width;
    double amp_c, width_c;
    int32_t is_point;
    int32_t pad;
    int64_t iter_added, iter_updated;
} asp_component;

/* Report of the last fit. members[0] = -1 is the new component, then the
 * indices of the refitted old components. */
typedef struct {
    int32_t n_active;
    int32_t members[ASP_MAX_ACTIVE];
    int32_t lm_iters;            /* LM trials used (both fits if a fallback ran) */
    int32_t converged;
    int32_t used_fallback;       /* the proposal's fit failed (no convergence or
                                    a zero amplitude); simple values fitted     */
    int64_t idx;                 /* peak pixel                                   */
    float peak;                  /* residual at the peak before the fit          */
    float pad;
    double chi2_init, chi2_final;/* sum over the fit's pixels of (D - M)^2       */
    double theta0[4 * ASP_MAX_ACTIVE];   /* start (a, x, y, s) per member        */
    double theta[4 * ASP_MAX_ACTIVE];    /* fitted, before the loop gain         */
    int64_t fit_px;              /* pixels in the union of windows at the fit    */
    int32_t init_source;         /* start values: 0 the simple values, 1 the
                                    caller's init, 2 the network, 3 the smoothing
                                    method (init holds its start)                */
    int32_t start_from_proposal; /* 1: the proposal scored a lower objective than
                                    the simple values and LM started from it     */
    double init[4];              /* the proposal (a, x, y, s) before clamping, or
                                    the smoothing method's start                 */
    int32_t added;               /* 1: the new component joined the list; 0: its
                                    fitted amplitude is zero (the old members
                                    explain the peak) and it was not added       */
    int32_t pad2;
} asp_fit_report;

typedef struct {
    int32_t struct_size;         /* sizeof(asp_options)                          */
    int32_t max_iter;            /* iteration count stop; default 1000           */
    int32_t max_active;          /* K_max, 1..ASP_MAX_ACTIVE; default 5          */
    int32_t lm_max_iter;         /* LM trial budget; default 100                 */
    int32_t init_mode;           /* 0 simple initial values, 1 learned proposal,
                                    2 the smoothing method with the 5 % switch  */
    int32_t capacity;            /* component list size; 0 = max_iter            */
    int32_t fit_solo_tiles;      /* LM trials over at most this many 256-pixel
                                    tiles are evaluated by one work-group;
                                    0 = default (16), -1 = never                 */
    int32_t fit_min_tiles;       /* least tiles per work-group when a trial is
                                    shared over the GPU; 0 = default (2)         */
    int32_t fit_group;           /* work-groups per first-level arrival counter of
                                    a shared trial; 0 = default (16)             */
    int32_t smooth_scales;       /* trial widths omega_b 2^j, j < smooth_scales,
                                    of the smoothing method, 1..ASP_MAX_SCALES;
                                    0 = default (5)                              */
    int32_t smooth_norm;         /* 0: the beams have peak 1 (default); 1: each
                                    smoothed value is divided by the L2 norm of
                                    the kernel on its clipped window             */
    int32_t switch_area;         /* areas compared by the switch: 0 pi s^2 of
                                    the fitted Gaussians (default); 1 the
                                    deconvolved pi (s^2 - omega_b^2)             */
    int32_t peak_tiles;          /* 0: the peak search scans the whole residual
                                    every iteration (default); 1: it keeps the
                                    maximum of |R| of every 64 x 64 tile on the
                                    device and rescans only the tiles that the
                                    residual updates touched (same result)      */
    int32_t refresh_every;       /* > 0: asp_run replaces the residual by the
                                    exact one (asp_refresh_residual) after every
                                    refresh_every-th iteration; 0 = never        */
    int32_t update_launch;       /* 0: in asp_run the residual update (Sect. 2
                                    step 3) runs at the end of the fit kernel,
                                    on all its work-groups (default); 1: its own
                                    kernel launch, as asp_update_residual does.
                                    Same result either way                       */
    int32_t reserved;            /* 0                                            */
    double window_sigmas;        /* window half-width factor c_w; default 5      */
    double max_width;            /* upper bound on s; 0 = max(omega_b, min(H,W)/8) */
    double lm_mu0;               /* initial damping; default 1e-3                */
    double lm_tol;               /* step tolerance; default 1e-5                 */
    double psf_lobe_frac;        /* main-lobe threshold; default 0.35            */
    void *stream;                /* hipStream_t to run on; NULL = own stream     */
} asp_options;

typedef struct {
    int64_t iterations;          /* iterations done by this call                 */
    int64_t total_iterations;    /* k after the call                             */
    int64_t components;          /* L after the call                             */
    int64_t lm_trials;           /* trials summed over this call's fits          */
    int64_t not_converged;       /* fits that used the whole budget              */
    int64_t fallbacks;           /* learned proposals replaced by simple values  */
    int64_t pixels_updated;      /* pixels read-modify-written by the updates    */
    int64_t pixels_evaluated;    /* pixel evaluations summed over the LM trials  */
    int64_t gram_flops;          /* (n+1)(n+2) per pixel evaluation: the FP32
                                    multiply-adds of [J r]^T [J r], n = 4 m      */
    int64_t smoothed;            /* fits started from the smoothing method       */
    int64_t peak_tiles_scanned;  /* 64 x 64 tiles rescanned by the incremental
                                    peak search (peak_tiles = 1)                 */
    int64_t not_added;           /* fits whose new component had amplitude zero
                                    and was not added                            */
} asp_run_report;

/* Fill *opt with the defaults above. */
asp_status asp_default_options(asp_options *opt);

/*
 * Create a context (Sect. 2, Eq. 1: dirty = PSF (*) sky + noise).
 *   dirty  H x W host image; psf Hp x Wp host image with its peak anywhere.
 *   gain   loop gain in (0, 1] (Sect. 3); threshold >= 0 (Sect. 2 step 4).
 *   opt    NULL for defaults.
 * Copies both images to the device, checks them for NaN/Inf
 * (ASP_ERR_NONFINITE), fits the Gaussian main lobe of the PSF on the device
 * (alpha_b, omega_b; Sect. 3) and allocates the component list.  On error
 * *out is NULL.
 */
asp_status asp_create(const float *dirty, int64_t H, int64_t W,
                      const float *psf, int64_t Hp, int64_t Wp,
                      float gain, float threshold, const asp_options *opt, asp_ctx **out);

/* As asp_create with device pointers (e.g. torch tensors); the images are
 * copied device to device on the context's stream. */
asp_status asp_create_device(const float *dirty_dev, int64_t H, int64_t W,
                             const float *psf_dev, int64_t Hp, int64_t Wp,
                             float gain, float threshold, const asp_options *opt,
                             asp_ctx **out);

void asp_destroy(asp_ctx *ctx);
const char *asp_last_error(const asp_ctx *ctx);

/*
 * Step 1-2 (Sect. 2 steps 1 and 4): the peak of |residual|, the lowest
 * row-major index winning ties, and the stop test.  Returns ASP_OK,
 * ASP_STOP_THRESHOLD or ASP_STOP_MAXITER.  idx and value may be NULL.
 */
asp_status asp_find_peak(asp_ctx *ctx, int64_t *idx, float *value);

/*
 * Step 3 (Sect. 3, Eq. 4): select the active set around pixel idx and fit it
 * by LM on the device.  init = NULL uses the simple initial values (the
 * residual at idx and the main-lobe width), or the network's proposal in
 * learned mode; otherwise init is a proposal in convolved space (clamped to
 * the peak's sign, s >= omega_b and 16 px of the peak).  With a proposal the
 * objective is evaluated at it and at the simple values and LM starts from the
 * lower; if it started from the proposal and does not converge, or converges
 * to a new component of amplitude zero, the simple values are fitted instead.
 * The active set depends on idx and the component
 * list only.  Must follow asp_find_peak.  rep may be NULL.  Returns ASP_OK or
 * ASP_LM_NOT_CONVERGED.
 */
asp_status asp_fit_active_set(asp_ctx *ctx, int64_t idx, const asp_gauss *init,
                              asp_fit_report *rep);

/*
 * Step 4 (Sect. 3 loop gain; Sect. 2 step 3 with the Gaussian beam): the fit's
 * commit, made on the device at the end of asp_fit_active_set, changes the
 * model by the loop gain times the fitted change -- the new component joins
 * with gain times its fitted amplitude (not at all when that amplitude is
 * zero), each old member moves the fraction gain of the way to its refit --
 * and this call updates the residual on the windows involved.  Must follow
 * asp_fit_active_set.  pixels_touched (nullable) receives the read-modify-
 * written pixel count.
 */
asp_status asp_update_residual(asp_ctx *ctx, int64_t *pixels_touched);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the peak
 * search of asp_find_peak (the largest |R|, the lowest row-major index on
 * ties) over a caller's image, with no context and no allocation.
 *   R          device image H x W, row-major FP32, 16-byte aligned; read only.
 *   idx_out    device int64: the peak pixel r W + c.
 *   value_out  device float: R at that pixel.
 *   stream     the HIP stream (NULL: the null stream); the call is
 *              asynchronous and may be captured into a graph.
 * Its scratch (64 packed keys, 512 bytes) is a file-scope device array, one
 * copy per GPU, held until the process ends; the call clears it with a
 * kernel before every scan.  Calls that overlap on one GPU (other streams,
 * other threads) share that array and race.  Returns ASP_ERR_INVALID_ARG for
 * null pointers, H or W < 1, H W >= 2^32 - 1 (the maximum: the key holds a
 * 32-bit index) or an unaligned image, with a message on stderr for the
 * last two; ASP_ERR_DEVICE when a launch fails.  No hipMalloc, hipFree or
 * allocating library call is made.
 */
asp_status asp_find_peak_noalloc(const float *R, int64_t H, int64_t W, int64_t *idx_out,
                                 float *value_out, void *stream);

/*
 * One evaluation of the fit objective on the device, the LM trial's own code
 * path (diagnostic; Sect. 3, Eq. 4 over the union U of the members' windows):
 * the m members' parameters theta (4 m doubles, (a, x, y, s), the new
 * component first) are evaluated against the context's residual with the
 * old members' stored Gaussians, stored[4 j .. 4 j + 3] for j >= 1, added
 * back on their stored windows (stored may be NULL when m = 1; stored[0..3]
 * is not read).  Outputs (host, each nullable): jtj = J^T J (n x n, n = 4 m,
 * row-major), jtr = J^T (D - M) (n), F = sum_U M (M - 2 D), chi2 =
 * sum_U (D - M)^2, npx = |U|.  Nothing of the context changes.  Returns
 * ASP_ERR_INVALID_ARG for m outside 1..ASP_MAX_ACTIVE or non-finite
 * parameters or widths that are not positive, ASP_ERR_STATE inside a
 * step-API sequence.
 */
asp_status asp_eval_trial(asp_ctx *ctx, int32_t m, const double *theta, const double *stored,
                          double *jtj, double *jtr, double *F, double *chi2, int64_t *npx);

/*
 * The report of the last fit made by any path (the step API, asp_step,
 * asp_run or a batched launch), read from the device state.  rep must not be
 * NULL.
 */
asp_status asp_last_fit(asp_ctx *ctx, asp_fit_report *rep);

/* One full iteration (find_peak, fit, update) without host round trips; the
 * update runs as in asp_run. */
asp_status asp_step(asp_ctx *ctx);

/*
 * Up to n_iter iterations on the device.  Iterations are queued in chunks
 * with no host synchronisation inside a chunk; every kernel checks the
 * device stop flag, so the run stops exactly where the stop test fires.
 * With update_launch 0 (the default) the residual update is done by the fit
 * kernel's work-groups after the commit, in the same launch; with 1 it is a
 * launch of its own.  The residual is the same bit for bit either way.
 * Returns ASP_OK (n_iter done), ASP_STOP_THRESHOLD or ASP_STOP_MAXITER.
 * rep may be NULL.
 */
asp_status asp_run(asp_ctx *ctx, int64_t n_iter, asp_run_report *rep);

/*
 * The component list with Eqs. 5-6 applied on the device.  Fills
 * min(cap, L) entries; *n = L.  Returns ASP_ERR_CAPACITY if cap < L.
 */
asp_status asp_components(asp_ctx *ctx, asp_component *out, int64_t cap, int64_t *n);

/* Raw convolved-space component list (a, x, y, s per row), FP64. */
asp_status asp_components_raw(asp_ctx *ctx, double *out4, int64_t cap, int64_t *n);

/* Copy the residual to a host buffer of H*W floats. */
asp_status asp_residual(asp_ctx *ctx, float *out);
/* Sum over the image of residual^2, in FP64 and a fixed order, on the
 * device (no copy of the image).  The full pass also re-bases the tracked
 * sum below. */
asp_status asp_residual_sumsq(asp_ctx *ctx, double *sum_sq);
/* The same sum, tracked without a pass over the image (for a noise-level stop
 * rule, Sect. 2 step 4): each windowed update (asp_update_residual, the steps
 * of asp_step / asp_run and of a batch) adds, per work-group, the FP64 change
 * sum(R_new^2 - R_old^2) over the pixels it rewrote into a slot of its own;
 * a full pass re-bases it at create, after every exact-PSF refresh, every
 * Asp-Clean2004 update, asp_load_state and asp_residual_sumsq.  The read adds
 * the base and the slots in a fixed order: deterministic, equal to the full
 * pass up to FP64 rounding; the error grows by about 2^-53 of the sum at the
 * last re-base per update (the per-pixel change is the difference of two
 * exact squares), so it is relative to that sum, not to the current one.  A
 * caller that writes the residual through asp_residual_device calls
 * asp_residual_sumsq afterwards to re-base.  *sum_sq (host) receives the sum;
 * ASP_ERR_INVALID_ARG for a null argument. */
asp_status asp_residual_sumsq_tracked(asp_ctx *ctx, double *sum_sq);
/* Device pointer of the residual (valid until asp_destroy). */
asp_status asp_residual_device(asp_ctx *ctx, float **dev);

/* The Gaussian fitted to the PSF main lobe (Sect. 3: alpha_b, omega_b). */
asp_status asp_psf_gauss(asp_ctx *ctx, double *alpha_b, double *omega_b);

/*
 * The model image of Sect. 2 step 2, I_model = sum of the components in the sky
 * plane (Eqs. 5-6), rendered as asp_refresh_residual renders it: a component
 * at least 1 px wide as its Gaussian sampled on the window of half-width
 * max(3, ceil(c_w omega)); a narrower one, points included, per axis by
 * three Gauss-Hermite nodes spread with the Lanczos-3 kernel and normalised.
 * Rendered in FP64 on the device; out receives H*W FP32 values (host buffer,
 * row-major).  The first call allocates the refresh's buffers and an H x W
 * device image.  Not available to batched fields.
 */
asp_status asp_model_image(asp_ctx *ctx, float *out);

/*
 * Checkpoint and resume.  The state is the residual, the component list, the
 * iteration count, the smoothing method's switch and the PSF's Gaussian
 * (alpha_b, omega_b): everything the next iteration depends on.  The options
 * and the input images are not part of it: load a state into a context
 * created from the same images, with the options the run should continue
 * under.  A stop is not part of it either: after a load the next iteration
 * applies the loading context's stop test.  Because every
 * reduction on the path has a fixed order, iterations after a load repeat
 * those of the run that saved the state, bit for bit.
 *   asp_state_size  bytes of the state blob now (64 + 4 H W + 48 L).
 *   asp_save_state  writes the blob into a host buffer of cap bytes; *bytes
 *                   (nullable) receives its size; ASP_ERR_CAPACITY when cap
 *                   is short.
 *   asp_load_state  restores a blob: ASP_ERR_INVALID_ARG when it is not a
 *                   state, has the wrong length, or comes from an image of
 *                   another size or another PSF fit; ASP_ERR_CAPACITY when its
 *                   list does not fit the context's capacity.
 * Both refuse to run inside a find_peak / fit / update sequence
 * (ASP_ERR_STATE); batched fields cannot load a state.
 */
asp_status asp_state_size(asp_ctx *ctx, int64_t *bytes);
asp_status asp_save_state(asp_ctx *ctx, void *blob, int64_t cap, int64_t *bytes);
asp_status asp_load_state(asp_ctx *ctx, const void *blob, int64_t bytes);

/* Iterations done (k) and components (L). */
asp_status asp_counts(asp_ctx *ctx, int64_t *k, int64_t *L);

/* Diagnostics: accumulated fit-kernel phase timers of the work-group that
 * drives the fit, in microseconds, then event counts; n <= 14 entries:
 * check-in, setup, evaluation, waits, reduction, LM step, commit, trial
 * preparation, arrival, then trials, fits, pixels evaluated, trials the
 * driving work-group evaluated alone and their pixels.  Reading does not
 * reset them. */
asp_status asp_fit_profile(asp_ctx *ctx, double *out, int32_t n);

/* Diagnostics: per active-set size m = 0 .. n - 1 (n <= ASP_MAX_ACTIVE + 1),
 * the fits that ended with m members, their LM trials and their device time
 * from the start values to the commit, in microseconds, summed since the
 * context was created.  Each pointer is nullable. */
asp_status asp_fit_histogram(asp_ctx *ctx, int64_t *fits, int64_t *trials, double *us, int32_t n);

/*
 * Learned start values.  A perceptron 1024 -> 256 -> 256 -> 4 (ReLU) maps the
 * 32 x 32 residual patch around the peak (rows r*-16..r*+15, columns
 * c*-16..c*+15, zero outside the image, divided by R[p*]) to
 * (a / R[p*], log(s / omega_b), x - c*, y - r*) of the new component, which
 * replaces the simple initial values of Sect. 3 as the start of the LM fit;
 * when that fit does not converge, or ends with a new component of amplitude
 * zero, the simple values are fitted instead.
 * Weights are FP32 in the order W1 (256 x 1024, row-major), b1, W2
 * (256 x 256), b2, W3 (4 x 256), b3: ASP_MLP_PARAMS values.
 */
#define ASP_MLP_PARAMS 329220
#define ASP_MLP_IN 1024
#define ASP_MLP_OUT 4

/* Give the context a network (host array of n = ASP_MLP_PARAMS floats,
 * copied). */
asp_status asp_set_mlp(asp_ctx *ctx, const float *weights, int64_t n);
/* 0: simple initial values; 1: the network (needs asp_set_mlp); 2: the
 * smoothing method with the switch (below). */
asp_status asp_set_init_mode(asp_ctx *ctx, int32_t mode);

/*
 * The smoothing method of initial values (Sect. 2 step 1; Sect. 3).  The
 * residual is smoothed with Gaussian beams of the trial widths
 * sigma_j = omega_b 2^j (j < smooth_scales, sigma_j not above the width bound
 * of the fit): C_j(p) is the sum over the window of half-width
 * max(3, ceil(c_w sigma_j)) around pixel p, clipped to the image, of
 * exp(-|q - p|^2 / (2 sigma_j^2)) R(q).  The peak among the smoothed images
 * is the largest |C_j(p)| (smooth_norm 0) or |C_j(p)| / sqrt(N_j(p)), N_j(p)
 * the sum of the squared kernel on the same window (smooth_norm 1); ties go
 * to the smaller j, then the smaller row-major p.  The new component then
 * starts at (C/N, x = column of p, y = row of p, s = sigma_j) -- the
 * least-squares amplitude of that Gaussian -- and the active set is selected
 * around that start.  In init mode 2 an iteration uses the smoothing method
 * unless the previous fit's new component had an area below 5 % of the area
 * of its start (switch_area); then the simple values are used.  The first
 * iteration smooths.  The smoothed images are kept on the device and
 * refreshed only where residual updates changed them.
 *
 * asp_smooth_peak: the smoothing method's peak on the current residual
 * (scale j, pixel, |score| as compared in FP32, start values in FP64; any
 * pointer may be NULL).  Needs no particular phase and leaves the iteration
 * state alone.  asp_smooth_map: the smoothed image of scale j (C_j, or
 * C_j / sqrt(N_j) with smooth_norm 1) as H*W floats into a host buffer.
 * asp_smooth_widths: the trial widths in use (n <= ASP_MAX_SCALES, fewer when
 * the width bound drops some).  Images with H W smooth_scales >= 2^32 - 1 are
 * refused (ASP_ERR_INVALID_ARG).
 */
#define ASP_MAX_SCALES 8
asp_status asp_smooth_peak(asp_ctx *ctx, int32_t *scale, int64_t *idx, float *score,
                           asp_gauss *start);
asp_status asp_smooth_map(asp_ctx *ctx, int32_t scale, float *out);
asp_status asp_smooth_widths(asp_ctx *ctx, double *sigma, int32_t cap, int32_t *n);
/*
 * Exact-PSF residual refresh (Sect. 2 step 3): R = I_dirty - B (*) I_model with
 * the true PSF B, instead of the residual the minor cycle keeps by subtracting
 * each component's Gaussian main-lobe approximation.  The model image holds
 * every component with its Eq. 5-6 parameters: components at least 1 px wide
 * as Gaussians sampled at pixel centres on the window of half-width
 * max(3, ceil(c_w omega)); narrower ones (points included) spread by
 * band-limited interpolation (per axis the 3-point Gauss-Hermite nodes of the
 * Gaussian, each with the Lanczos-3 kernel, weights normalised to sum 1).
 * The convolution is linear, zero outside the image, with the PSF centred on
 * its peak pixel, computed in FP64 through FFTs of a zero-padded grid; R is
 * rounded to FP32.  Needs no particular phase; the component list is kept.
 */
asp_status asp_refresh_residual(asp_ctx *ctx);

/*
 * The Asp-Clean2004 iteration, the comparison path of the paper (Sect. 2
 * steps 1-4 with the objective of Eq. 3; the cost count after it; Table 3).
 *   1. the peak of |residual| and the stop test, as asp_find_peak;
 *   2. start values from the smoothing method (every iteration; no switch),
 *      turned into sky-plane values by Eq. 5: omega_0^2 = max(s^2 -
 *      omega_b^2, 0), F_0 = a s^2 / (alpha_b omega_b^2);
 *   3. Levenberg-Marquardt fit of the one new component theta = (F, x, y,
 *      v = omega^2) against chi^2 = || R - B (*) g(theta) ||^2 over the whole
 *      image with the true PSF B, convolved in FP64 in every evaluation (by
 *      FFT or directly, asp_set_2004_convolution).  g is the unit-flux component rendered as
 *      asp_refresh_residual renders the model, times F; the squared width
 *      keeps the objective differentiable at a point source.  Bounds: F keeps
 *      the start's sign, x and y stay in the start's window,
 *      0 <= v <= s_max^2 - omega_b^2.  LM rules, budget (lm_max_iter) and
 *      tolerance are those of asp_fit_active_set;
 *   4. R -= gain B (*) g(theta) (exact, FP64, rounded to FP32), and the
 *      component joins the list as the convolved-space Gaussian whose Eqs. 5-6
 *      deconvolution is (gain F, omega), so asp_components and
 *      asp_refresh_residual read it like any other.
 * Earlier components are not refitted.  The host reads the device's LM state
 * after each evaluation (after every four on padded grids of at most 1024^2
 * pixels, where evaluations queued past the end of the fit return at once).
 * The first call allocates four FP64 grids and their spectra of the
 * refresh's padded size, the per-axis factors of the rendering and their 1-D
 * DFTs, and a batched inverse FFT plan.  Must not be
 * inside a find_peak / fit / update sequence (ASP_ERR_STATE); not available
 * to batched fields.  Returns ASP_OK, ASP_LM_NOT_CONVERGED (budget used),
 * ASP_STOP_THRESHOLD or ASP_STOP_MAXITER.  rep may be NULL.
 */
typedef struct {
    int64_t idx;                 /* peak pixel                                   */
    float peak;                  /* residual there before the fit                */
    int32_t scale;               /* trial width j of the smoothing start         */
    int32_t trials;              /* LM trials                                    */
    int32_t converged;
    int32_t evaluations;         /* evaluations of Eq. 3 (trials + the start)    */
    int32_t direct_evals;        /* of those, convolved directly (the rest by FFT)*/
    double start[4];             /* the smoothing start (a, x, y, s), convolved  */
    double theta0[4];            /* sky (F, x, y, omega^2) start in the bounds   */
    double theta[4];             /* fitted sky (F, x, y, omega^2), before gain   */
    double lo[4], hi[4];         /* the bounds                                   */
    double chi2_init, chi2_final;/* over the whole image                         */
    int32_t direct_update;       /* 1: the update was convolved directly         */
    int32_t pad;
} asp_fit2004_report;

/*
 * How asp_step_2004 and asp_run_2004 form B (*) g (Sect. 2 step 3 and Eq. 3
 * with the true PSF).  Every image the rendering makes is a sum of outer
 * products of per-axis factors, so B (*) g is also a pass along the rows of
 * the PSF with the column factors and one along the columns with the row
 * factors, in FP64, with the same result up to rounding; its cost grows with
 * the taps (12 per axis below omega = 1 px, 2 h + 1 above) where the FFTs'
 * does not.  mode 0 (default): directly when its multiply-adds undercut a
 * fixed count per padded FFT pixel, by the squared width of the point under
 * evaluation (or, on padded grids of at most 1024^2 pixels, where four
 * evaluations are queued per read, by its upper bound), else by FFT; 1: always
 * by FFT; 2: directly.  The direct row pass keeps (H + nr - 1) x W rows per
 * factor in the FFT grids (three factors for an evaluation, one for the
 * update); where they would not fit, the FFT is used in every mode.
 * ASP_ERR_INVALID_ARG for another mode.
 */
asp_status asp_set_2004_convolution(asp_ctx *ctx, int32_t mode);

asp_status asp_step_2004(asp_ctx *ctx, asp_fit2004_report *rep);

/* Up to n_iter Asp-Clean2004 iterations; rep as for asp_run (lm_trials,
 * not_converged, pixels_evaluated = evaluations x H x W, smoothed).  Returns
 * ASP_OK (n_iter done), ASP_STOP_THRESHOLD or ASP_STOP_MAXITER. */
asp_status asp_run_2004(asp_ctx *ctx, int64_t n_iter, asp_run_report *rep);

/* Work of the smoothing passes since the context was created: output pixels
 * inside the image summed over both passes and all scales, and the
 * multiply-adds they stand for, 2 (2 h_j + 1) flops per pixel of scale j. */
asp_status asp_smooth_work(asp_ctx *ctx, int64_t *pixels, double *flops);

/*
 * Record a training pair per iteration into caller-owned device buffers:
 * patches (cap x 1024 FP32, the network's input), targets (cap x 4 FP32, the
 * fitted new component before the loop gain, encoded as the network's
 * output) and flags (cap int32: bit 0 converged, bit 1 fallback used, bits
 * 2-3 init_source).  Recording covers asp_run, asp_step and the step API; it
 * stops when cap pairs are stored.  cap = 0 turns it off.  The buffers must
 * stay valid while recording is on.
 */
asp_status asp_record(asp_ctx *ctx, float *patches_dev, float *targets_dev, int32_t *flags_dev,
                      int64_t cap);
asp_status asp_record_count(asp_ctx *ctx, int64_t *n);

/*
 * Training on the device (forward and backward passes and Adam by the
 * library's own kernels, FP32).  The loss of a batch is the mean over samples
 * and outputs of (y - t)^2.
 *   asp_mlp_create    weights from a host array of ASP_MLP_PARAMS floats
 *                     (copied); batches of at most max_batch rows; stream NULL
 *                     = own stream.  Adam moments start at zero.
 *   asp_mlp_loss_grad loss and gradient of one batch (device x: batch x 1024,
 *                     t: batch x 4); grad (host, ASP_MLP_PARAMS, nullable)
 *                     is in the weights' order.  No update.
 *   asp_mlp_train     n_steps Adam steps (lr, beta1 0.9, beta2 0.999, eps
 *                     1e-8) on batches of `batch` rows of (x, t) (device,
 *                     n_rows rows each) picked by order (device int32,
 *                     n_steps x batch row indices; an index outside
 *                     [0, n_rows) is an ASP_ERR_INVALID_ARG); *mean_loss is
 *                     the mean batch loss.
 *   asp_mlp_forward   outputs (device, rows x 4) for device inputs rows x 1024.
 *   asp_mlp_weights   the current weights to a host array.
 */
typedef struct asp_mlp asp_mlp;
asp_status asp_mlp_create(const float *init, int32_t max_batch, void *stream, asp_mlp **out);
void asp_mlp_destroy(asp_mlp *net);
const char *asp_mlp_last_error(const asp_mlp *net);
asp_status asp_mlp_loss_grad(asp_mlp *net, const float *x_dev, const float *t_dev, int32_t batch,
                             double *loss, float *grad);
asp_status asp_mlp_train(asp_mlp *net, const float *x_dev, const float *t_dev, int64_t n_rows,
                         const int32_t *order_dev, int64_t n_steps, int32_t batch, float lr,
                         double *mean_loss);
asp_status asp_mlp_forward(asp_mlp *net, const float *x_dev, int64_t rows, float *y_dev);
asp_status asp_mlp_weights(asp_mlp *net, float *out);

/*
 * Batched fields: many independent fields deconvolved by one persistent
 * launch, captured in a HIP graph and replayed.  Each field is an ordinary
 * context (asp_batch_field; every single-field call works on it between
 * runs); its minor cycle is the one of asp_run.  The launch fills the GPU
 * with work-groups grouped in teams of team_size on one XCD each; a team takes
 * fields from a queue (largest first) and runs each for n_iter iterations or
 * until it stops.
 *   asp_batch_create   fields i = 0..n_fields-1 from host arrays, as
 *                      asp_create with gain[i], threshold[i]; opt (NULL =
 *                      defaults) applies to all; opt->stream must be NULL.
 *   asp_batch_config   team_size (work-groups per team; must divide the
 *                      work-groups of one XCD), solo_tiles, min_tiles as in
 *                      asp_options; 0 keeps a value.
 *   asp_batch_run      one launch: up to n_iter iterations per field.  rep:
 *                      iterations summed over fields, fields stopped, fields
 *                      failed, device milliseconds of the launch.
 *   asp_batch_autotune coordinate search over team size, solo_tiles and
 *                      min_tiles on real chunks of probe_iter iterations per
 *                      field (the fields advance); applies and returns the
 *                      fastest.
 * A batch is not thread-safe; its contexts must not be used while it runs.
 */
typedef struct asp_batch asp_batch;
typedef struct {
    int64_t iterations;
    int64_t fields_stopped;
    int64_t fields_failed;
    double ms;
} asp_batch_report;
asp_status asp_batch_create(int32_t n_fields, const float *const *dirty, const int64_t *H,
                            const int64_t *W, const float *const *psf, const int64_t *Hp,
                            const int64_t *Wp, const float *gain, const float *threshold,
                            const asp_options *opt, asp_batch **out);
void asp_batch_destroy(asp_batch *batch);
const char *asp_batch_last_error(const asp_batch *batch);
asp_status asp_batch_field(asp_batch *batch, int32_t i, asp_ctx **ctx);
asp_status asp_batch_config(asp_batch *batch, int32_t team_size, int32_t solo_tiles,
                            int32_t min_tiles);
asp_status asp_batch_get_config(asp_batch *batch, int32_t *team_size, int32_t *solo_tiles,
                                int32_t *min_tiles, int32_t *grid);
asp_status asp_batch_run(asp_batch *batch, int64_t n_iter, asp_batch_report *rep);
asp_status asp_batch_autotune(asp_batch *batch, int64_t probe_iter, int32_t *team_size,
                              int32_t *solo_tiles, int32_t *min_tiles);

/* Diagnostics: per-kernel device time.  With timing on, asp_run, asp_step,
 * asp_smooth_peak, asp_refresh_residual, asp_step_2004 and asp_run_2004
 * record a HIP event pair on the context's stream around every launch they
 * make (which adds two event packets per launch); asp_kernel_times returns
 * the summed milliseconds and launch counts, n <= 9 kinds: 0 peak search,
 * 1 LM fit, 2 residual update, 3 proposal / patch recording, 4 the smoothing
 * passes (column and row pass together), 5 the smoothing pick, 6 the
 * exact-PSF refresh (rendering, two FFTs, spectral product, subtraction),
 * 7 one evaluation of the Asp-Clean2004 objective (rendering of the component
 * and its derivatives with the batched FFTs, or the factors with the two
 * direct passes; the sums, the LM decision; queued evaluations past the end
 * of a fit included), 8 the Asp-Clean2004 update (the convolution of either
 * kind, subtraction, the new component).
 * Switching timing on or off clears the totals. */
asp_status asp_kernel_timing(asp_ctx *ctx, int32_t on);
asp_status asp_kernel_times(asp_ctx *ctx, double *ms, int64_t *launches, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* ASP_H */
