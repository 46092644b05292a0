/*
 * FP64 CPU oracle of the Asp-Clean2016 minor cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * What it computes (Zhang, Bhatnagar, Rau & Zhang 2016, "Efficient
 * implementation of the adaptive scale pixel decomposition algorithm"):
 *   - Sect. 2, Eq. (1)/(2): dirty = PSF (*) sky + noise, sky = sum of components.
 *   - Sect. 2, the Asp-Clean loop (steps 1-4): find the peak, fit, update the
 *     residual, repeat until an iteration count or a threshold stops it.
 *   - Sect. 3, Eq. (4): each fit minimises || residual - Gaussian ||^2 with the
 *     PSF-convolved component written as an analytic Gaussian (no FFT).
 *   - Sect. 3, Eqs. (5)-(6): the component is recovered from the fitted
 *     Gaussian by analytic deconvolution of the Gaussian main lobe.
 *   - Sect. 3: a loop gain scales the new component before it joins the model;
 *     read here as scaling every change of the model image, so a refitted old
 *     member of the active set moves the fraction gain toward its refit.
 *   - Sect. 3: the simple initial values (the residual peak and the main-lobe
 *     width of the PSF).
 * Readings where the paper is silent (active set, windows, LM constants) are
 * listed in the repository's design notes and restated at each function.
 *
 * Conventions: images are row-major, pixel (r, c) at index r*W + c, pixel
 * centres at integer coordinates, x = column, y = row.  A Gaussian component
 * in convolved ("fit") space is (a, x, y, s): a * exp(-((c-x)^2+(r-y)^2)/(2 s^2)),
 * point-sampled at pixel centres; s is the standard deviation (the width
 * omega of Sect. 3 enters the exponent as 1/(2 omega^2)).
 */
#ifndef ASP_ORACLE_H
#define ASP_ORACLE_H
#include <stdint.h>

#define ORC_MAX_ACTIVE 16

typedef struct {
    double a, x, y, s;          /* convolved-space Gaussian                   */
    int64_t iter_added;         /* iteration that created the component       */
    int64_t iter_updated;       /* last iteration that (re)fitted it          */
} orc_comp;

typedef struct {
    /* configuration */
    int64_t H, W;
    double gain, threshold;
    int64_t max_iter;
    int32_t max_active;         /* K_max: new component + refitted old ones   */
    int32_t lm_max_iter;        /* LM trial budget T_max                      */
    double max_width;           /* upper bound on s; 0 = max(omega_b, min(H,W)/8) */
    double window_sigmas;       /* window half-width factor c_w               */
    double lm_mu0, lm_tol;
    double alpha_b, omega_b;    /* Gaussian fitted to the PSF main lobe       */
    /* state (buffers owned by the caller) */
    double *R;                  /* residual, H*W                              */
    orc_comp *comps;            /* component list, capacity cap               */
    int64_t L, cap;
    int64_t k;                  /* iterations done                            */
} orc_state;

typedef struct {
    int32_t status;             /* ORC_OK / ORC_STOP_* / ORC_LM_NOT_CONVERGED / <0 error */
    int32_t n_active;
    int64_t idx;                /* peak pixel                                 */
    double peak;                /* R[idx] before the step                     */
    int32_t members[ORC_MAX_ACTIVE];  /* -1 = the new component, else index   */
    int32_t lm_iters, converged, used_fallback;
    int32_t start_from_proposal; /* LM started from the proposal (it scored lower) */
    double chi2_init, chi2_final;
    double theta[4 * ORC_MAX_ACTIVE]; /* fitted (a,x,y,s) per member, before the
                                         loop gain moves the list toward it     */
    double theta0[4 * ORC_MAX_ACTIVE];/* starting point of the fit            */
    int64_t omega_px;           /* pixels of U(theta) at the fitted theta     */
    int64_t update_px;          /* pixels read-modify-written by the update   */
    int32_t added;              /* 1: the new component joined the list (its   */
    int32_t pad;                /*    fitted amplitude is not zero)            */
} orc_report;

enum { ORC_OK = 0, ORC_STOP_THRESHOLD = 1, ORC_STOP_MAXITER = 2, ORC_LM_NOT_CONVERGED = 3,
       ORC_ERR_ARG = -1, ORC_ERR_NONFINITE = -2, ORC_ERR_PSF = -3, ORC_ERR_CAPACITY = -5 };

/* Defaults of the readings: c_w = 5, T_max = 50, mu0 = 1e-3, step tolerance
 * 1e-5. */
void orc_default_config(orc_state *st);

int orc_halfwidth(double s, double window_sigmas);
/* Window of half-width h centred on (floor(x+0.5), floor(y+0.5)), clipped to
 * the image; box = {r0, r1, c0, c1} inclusive.  Returns 0 if empty. */
int orc_box(double x, double y, int h, int64_t H, int64_t W, int64_t box[4]);

/* Row-major argmax of |R|, the lowest index winning ties. */
int64_t orc_peak(const double *R, int64_t n);

/* Circular Gaussian fitted to the PSF main lobe (centre at the PSF peak). */
int orc_psf_fit(const double *psf, int64_t Hp, int64_t Wp, double main_lobe_frac,
                double *alpha_b, double *omega_b, int64_t *n_lobe_px);

/* Eq. (5)/(6): deconvolve a fitted Gaussian (a, s) by the beam (alpha_b,
 * omega_b).  flux = 2 pi alpha omega^2 = a s^2 / (alpha_b omega_b^2). */
void orc_deconvolve(double a, double s, double alpha_b, double omega_b,
                    double *flux, double *alpha, double *omega, int32_t *is_point);
/* The forward direction: a sky Gaussian (alpha, omega) convolved with the beam. */
void orc_convolve(double alpha, double omega, double alpha_b, double omega_b,
                  double *a, double *s);

/* Dense SPD solve by Cholesky: A (n x n, row-major, not modified) x = b.
 * Returns 0, or -1 when A is not numerically positive definite. */
int orc_cholesky_solve(int n, const double *A, const double *b, double *x);

/* One minor-cycle iteration from the given state (peak, stop test, initial
 * values, active set, LM fit, commit, residual update).  init = NULL for the
 * simple initial values; otherwise a proposal (a, x, y, s) that is clamped and
 * falls back to the simple values when its fit does not converge.  hess_out
 * (nullable) receives the final J^T J (n x n, n = 4 * n_active). */
int orc_step(orc_state *st, const double *init, orc_report *rep, double *hess_out);

/* One iteration whose new component starts at start4 = (a, x, y, s), the
 * start values of the smoothing method (Sect. 2 step 1, Sect. 3), computed by
 * the caller.  The peak and the stop test are those of orc_step; the active
 * set is selected around start4 (sign of a, window of half-width h(s) around
 * (x, y), co-location radius max(omega_b, min(s_j, s))); no fallback. */
int orc_step_start(orc_state *st, const double *start4, orc_report *rep, double *hess_out);

/* Up to n_iter iterations of orc_step with the simple initial values; returns
 * the last status and the number of iterations done. */
int orc_run(orc_state *st, int64_t n_iter, int64_t *done);

/* out = dirty - sum_j G_j on W_j  (the residual from its definition). */
void orc_residual_from_scratch(const orc_state *st, const double *dirty, double *out);

/* One evaluation of the fit objective (Eq. 4 on the union U of the members'
 * windows, the data being R with the old members' stored Gaussians added back
 * on their stored windows): returns F = sum_U M (M - 2 D); H (n x n, n = 4 m,
 * nullable) = J^T J, g (n, nullable) = J^T (D - M), chi2 (nullable) =
 * sum_U (D - M)^2, npx (nullable) = |U|.  theta holds the m members' (a, x,
 * y, s), the new component first; stored[4 j .. 4 j + 3] the stored
 * parameters of old member j >= 1 (stored[0..3] unused).  Data: st->R. */
double orc_fit_eval(const orc_state *st, int m, const double *theta, const double *stored,
                    double *H, double *g, double *chi2, int64_t *npx);

/* One LM fit of m Gaussians (theta, updated in place) to a data image with no
 * add-back of old components, by the same objective and LM as orc_step.
 * Returns the trials used. */
int orc_fit_gaussians(const double *data, int64_t H, int64_t W, int m, double *theta,
                      double omega_b, double max_width, double window_sigmas, int lm_max_iter,
                      double mu0, double tol, int32_t *converged, double *chi2);

#endif
