/*
 * FP64 CPU oracle of the Asp-Clean2016 minor cycle.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the HIP library.  Plain, slow, single-threaded FP64 C written from
 * the paper (Sect. 2 loop, Sect. 3 Eqs. 4-6); see asp_oracle.h.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared asp_oracle.c -lm
 * (no fast-math; no fused multiply-add, so every FP64 expression rounds the
 * way it is written).
 */
#include "asp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

void orc_default_config(orc_state *st)
{
    st->gain = 0.1;
    st->threshold = 0.0;
    st->max_iter = 1000;
    st->max_active = 5;
    st->lm_max_iter = 100;
    st->max_width = 0.0;
    st->window_sigmas = 5.0;
    st->lm_mu0 = 1e-3;
    st->lm_tol = 1e-5;
    st->alpha_b = 1.0;
    st->omega_b = 1.0;
    st->L = 0;
    st->k = 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry.  The paper's norm runs over the image (Eq. 4); a window bounds   */
/* where a Gaussian is evaluated.  Reading: half-width h(s) = max(3,          */
/* ceil(c_w s)) around the rounded centre, clipped to the image.              */
/* ------------------------------------------------------------------------ */

int orc_halfwidth(double s, double window_sigmas)
{
    double h = ceil(window_sigmas * s);
    if (!(h >= 3.0)) h = 3.0;          /* also catches NaN */
    if (h > 1073741823.0) h = 1073741823.0;
    return (int)h;
}

int orc_box(double x, double y, int h, int64_t H, int64_t W, int64_t box[4])
{
    int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
    int64_t r0 = cy - h, r1 = cy + h, c0 = cx - h, c1 = cx + h;
    if (r0 < 0) r0 = 0;
    if (c0 < 0) c0 = 0;
    if (r1 > H - 1) r1 = H - 1;
    if (c1 > W - 1) c1 = W - 1;
    box[0] = r0; box[1] = r1; box[2] = c0; box[3] = c1;
    return (r0 <= r1 && c0 <= c1);
}

static int in_box(const int64_t b[4], int64_t r, int64_t c)
{
    return r >= b[0] && r <= b[1] && c >= b[2] && c <= b[3];
}

static void comp_window(const orc_state *st, double x, double y, double s, int64_t box[4])
{
    orc_box(x, y, orc_halfwidth(s, st->window_sigmas), st->H, st->W, box);
}

static double gauss_at(double a, double x, double y, double s, int64_t r, int64_t c)
{
    double dx = (double)c - x, dy = (double)r - y;
    return a * exp(-(dx * dx + dy * dy) / (2.0 * s * s));
}

/* ------------------------------------------------------------------------ */
/* Peak search (Sect. 2 step 1 with the simple method of Sect. 3): largest   */
/* |R|, lowest row-major index on ties.                                      */
/* ------------------------------------------------------------------------ */

int64_t orc_peak(const double *R, int64_t n)
{
    int64_t best = 0;
    double bv = -1.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = fabs(R[i]);
        if (v > bv) { bv = v; best = i; }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Dense Cholesky solve (textbook, row-major).                               */
/* ------------------------------------------------------------------------ */

int orc_cholesky_solve(int n, const double *A, const double *b, double *x)
{
    double *Lm = (double *)calloc((size_t)n * n, sizeof(double));
    if (!Lm) return -1;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double sum = A[i * n + j];
            for (int k = 0; k < j; ++k) sum -= Lm[i * n + k] * Lm[j * n + k];
            if (i == j) {
                if (!(sum > 0.0) || !isfinite(sum)) { free(Lm); return -1; }
                Lm[i * n + i] = sqrt(sum);
            } else {
                Lm[i * n + j] = sum / Lm[j * n + j];
            }
        }
    }
    /* L y = b */
    for (int i = 0; i < n; ++i) {
        double sum = b[i];
        for (int k = 0; k < i; ++k) sum -= Lm[i * n + k] * x[k];
        x[i] = sum / Lm[i * n + i];
    }
    /* L^T x = y */
    for (int i = n - 1; i >= 0; --i) {
        double sum = x[i];
        for (int k = i + 1; k < n; ++k) sum -= Lm[k * n + i] * x[k];
        x[i] = sum / Lm[i * n + i];
    }
    free(Lm);
    for (int i = 0; i < n; ++i)
        if (!isfinite(x[i])) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eqs. (5)/(6): analytic deconvolution of the Gaussian main lobe.           */
/*   omega_i^2 = omega_ic^2 - omega_b^2                          (Eq. 5)    */
/*   alpha_i   = alpha_ic omega_ic^2 / (2 pi alpha_b omega_b^2 omega_i^2)     */
/*                                                               (Eq. 6)    */
/* The flux 2 pi alpha_i omega_i^2 = alpha_ic omega_ic^2 / (alpha_b          */
/* omega_b^2) stays finite as omega_i -> 0 (an unresolved component).        */
/* ------------------------------------------------------------------------ */

void orc_deconvolve(double a, double s, double alpha_b, double omega_b,
                    double *flux, double *alpha, double *omega, int32_t *is_point)
{
    double w2 = s * s - omega_b * omega_b;
    if (w2 < 0.0) w2 = 0.0;
    double w = sqrt(w2);
    *flux = a * s * s / (alpha_b * omega_b * omega_b);
    *omega = w;
    if (w > 1e-6 * omega_b) {
        *alpha = a * s * s / (2.0 * ORC_PI * alpha_b * omega_b * omega_b * w2);
        *is_point = 0;
    } else {
        *alpha = 0.0;
        *is_point = 1;
    }
}

void orc_convolve(double alpha, double omega, double alpha_b, double omega_b,
                  double *a, double *s)
{
    double s2 = omega * omega + omega_b * omega_b;
    *s = sqrt(s2);
    *a = 2.0 * ORC_PI * alpha * alpha_b * omega * omega * omega_b * omega_b / s2;
}

/* ------------------------------------------------------------------------ */
/* The objective of Eq. (4) over the whole image.                            */
/*                                                                           */
/* Each member j of the fit is a Gaussian truncated to its window W(theta_j) */
/* (half-width h(s_j) around its rounded centre), so the model M is zero     */
/* outside U(theta) = union of the members' windows and                      */
/*   sum_image (D - M)^2 = sum_image D^2 + sum_{U(theta)} M (M - 2 D).       */
/* The first term does not depend on theta; the fit minimises the second,    */
/* F(theta), enumerating U(theta) window by window with pixels of earlier    */
/* windows skipped.  The windows move with theta.  The data are              */
/* D = R + sum_old G(theta_old)[W(theta_old)]: the residual with the old     */
/* members of the active set added back, so that the update afterwards       */
/* changes exactly the pixels the fit accounted for.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_state *st;
    int m;                               /* members; 0 = the new component    */
    double old[4 * ORC_MAX_ACTIVE];      /* stored parameters of old members  */
    int64_t wold[ORC_MAX_ACTIVE][4];     /* their stored windows              */
    const double *data;                  /* plain data image (no add-back)    */
    double lo[4 * ORC_MAX_ACTIVE], hi[4 * ORC_MAX_ACTIVE];
} fit_problem;

/* Data value D at pixel (r, c). */
static double fit_data(const fit_problem *fp, int64_t r, int64_t c)
{
    double d = fp->data[r * fp->st->W + c];
    for (int j = 1; j < fp->m; ++j)
        if (in_box(fp->wold[j], r, c))
            d += gauss_at(fp->old[4 * j], fp->old[4 * j + 1], fp->old[4 * j + 2],
                          fp->old[4 * j + 3], r, c);
    return d;
}

/* F(theta) = sum_{U(theta)} M (M - 2 D);  Hs = J^T J,  g = J^T (D - M), with
 * J = dM/dtheta.  Per member (a, x, y, s): dM/da = e, dM/dx = G (c - x)/s^2,
 * dM/dy = G (r - y)/s^2, dM/ds = G q / s^3, G = a e, e = exp(-q / (2 s^2)).
 * chi2 (nullable) receives sum_{U(theta)} (D - M)^2; npx the size of U. */
static double fit_eval(const fit_problem *fp, const double *theta, double *Hs, double *g,
                       double *chi2, int64_t *npx)
{
    const orc_state *st = fp->st;
    int m = fp->m, n = 4 * m;
    int64_t win[ORC_MAX_ACTIVE][4];
    for (int j = 0; j < m; ++j)
        comp_window(st, theta[4 * j + 1], theta[4 * j + 2], theta[4 * j + 3], win[j]);
    if (Hs) memset(Hs, 0, sizeof(double) * (size_t)n * n);
    if (g) memset(g, 0, sizeof(double) * (size_t)n);
    double F = 0.0, X = 0.0;
    int64_t count = 0;
    double Jrow[4 * ORC_MAX_ACTIVE];
    int cov[ORC_MAX_ACTIVE];
    for (int w = 0; w < m; ++w)
        for (int64_t r = win[w][0]; r <= win[w][1]; ++r)
            for (int64_t c = win[w][2]; c <= win[w][3]; ++c) {
                int seen = 0;
                for (int i = 0; i < w && !seen; ++i) seen = in_box(win[i], r, c);
                if (seen) continue;
                ++count;
                double M = 0.0;
                int nc = 0;
                for (int j = 0; j < m; ++j) {
                    if (!in_box(win[j], r, c)) continue;
                    const double *t = theta + 4 * j;
                    double dx = (double)c - t[1], dy = (double)r - t[2];
                    double q = dx * dx + dy * dy;
                    double s2 = t[3] * t[3];
                    double e = exp(-q / (2.0 * s2));
                    double G = t[0] * e;
                    M += G;
                    Jrow[4 * j + 0] = e;
                    Jrow[4 * j + 1] = G * dx / s2;
                    Jrow[4 * j + 2] = G * dy / s2;
                    Jrow[4 * j + 3] = G * q / (s2 * t[3]);
                    cov[nc++] = j;
                }
                double D = fit_data(fp, r, c);
                double res = D - M;
                F += M * (M - 2.0 * D);
                X += res * res;
                if (!Hs) continue;
                for (int u = 0; u < nc; ++u)
                    for (int a = 0; a < 4; ++a) {
                        int i = 4 * cov[u] + a;
                        g[i] += Jrow[i] * res;
                        for (int v = u; v < nc; ++v)
                            for (int b = 0; b < 4; ++b) {
                                int k = 4 * cov[v] + b;
                                if (k < i) continue;
                                Hs[i * n + k] += Jrow[i] * Jrow[k];
                            }
                    }
            }
    if (Hs)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < i; ++k) Hs[i * n + k] = Hs[k * n + i];
    if (chi2) *chi2 = X;
    if (npx) *npx = count;
    return F;
}

double orc_fit_eval(const orc_state *st, int m, const double *theta, const double *stored,
                    double *H, double *g, double *chi2, int64_t *npx)
{
    if (m < 1 || m > ORC_MAX_ACTIVE) return NAN;
    fit_problem fp;
    memset(&fp, 0, sizeof fp);
    fp.st = st;
    fp.m = m;
    fp.data = st->R;
    for (int j = 1; j < m; ++j) {
        memcpy(fp.old + 4 * j, stored + 4 * j, 4 * sizeof(double));
        comp_window(st, stored[4 * j + 1], stored[4 * j + 2], stored[4 * j + 3], fp.wold[j]);
    }
    return fit_eval(&fp, theta, H, g, chi2, npx);
}

/* ------------------------------------------------------------------------ */
/* Levenberg-Marquardt (Marquardt 1963), as used in Sect. 3 for Eq. (4).     */
/* Readings: the damped system (H + mu D) delta = g with                     */
/* D = diag(max(H_ii, 1e-12 max H_ii)); mu0 = 1e-3; a parameter on a bound   */
/* whose gradient points out of the box is held fixed for that trial (its    */
/* row and column become the identity, its right-hand side 0) and the trial  */
/* point is clipped to the bounds; a trial is accepted iff F decreases.  The */
/* damping follows the gain ratio rho = (F - F_trial) / (delta^T (g + mu D  */
/* delta)) (Madsen, Nielsen & Tingleff 2004): on accept mu *= max(1/3,       */
/* 1 - (2 rho - 1)^3) and nu = 2, on reject mu *= nu and nu *= 2; mu is kept */
/* in [1e-12, 1e8].  Converged when an accepted step has                     */
/* max |delta_k| / scale_k < tol (scale |a| for a, s for x, y, s); stalled   */
/* (treated as converged) once a rejection pushes mu past 1e8; the budget    */
/* counts trials.                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int trials, converged;
    double F0, F, chi2_0, chi2;
    int64_t npx;
} lm_result;

static void clip_to(double *theta, int n, const double *lo, const double *hi)
{
    for (int i = 0; i < n; ++i) {
        if (!(theta[i] >= lo[i])) theta[i] = lo[i];
        if (theta[i] > hi[i]) theta[i] = hi[i];
    }
}

static lm_result lm_fit(const fit_problem *fp, double *theta, int budget, double mu0,
                        double tol, double *hess_out)
{
    int m = fp->m, n = 4 * m;
    double *Hs = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *Ht = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double g[4 * ORC_MAX_ACTIVE], gt[4 * ORC_MAX_ACTIVE], delta[4 * ORC_MAX_ACTIVE];
    double rhs[4 * ORC_MAX_ACTIVE], trial[4 * ORC_MAX_ACTIVE], dd[4 * ORC_MAX_ACTIVE];
    lm_result res = {0, 0, 0.0, 0.0, 0.0, 0.0, 0};

    clip_to(theta, n, fp->lo, fp->hi);
    double F = fit_eval(fp, theta, Hs, g, &res.chi2_0, NULL);
    double chi2 = res.chi2_0;
    res.F0 = F;
    double mu = mu0, nu = 2.0;
    while (res.trials < budget) {
        double dmax = 0.0;
        for (int i = 0; i < n; ++i)
            if (Hs[i * n + i] > dmax) dmax = Hs[i * n + i];
        memcpy(A, Hs, sizeof(double) * (size_t)n * n);
        memcpy(rhs, g, sizeof(double) * (size_t)n);
        for (int i = 0; i < n; ++i) {
            dd[i] = Hs[i * n + i];
            if (dd[i] < 1e-12 * dmax) dd[i] = 1e-12 * dmax;
            A[i * n + i] += mu * dd[i];
        }
        for (int i = 0; i < n; ++i) {
            if ((theta[i] <= fp->lo[i] && g[i] <= 0.0) || (theta[i] >= fp->hi[i] && g[i] >= 0.0)) {
                for (int k = 0; k < n; ++k) { A[i * n + k] = 0.0; A[k * n + i] = 0.0; }
                A[i * n + i] = 1.0;
                rhs[i] = 0.0;
            }
        }
        res.trials++;
        int ok = orc_cholesky_solve(n, A, rhs, delta) == 0;
        double Ft = INFINITY, pred = 0.0, chi2t = 0.0;
        if (ok) {
            for (int i = 0; i < n; ++i) {
                trial[i] = theta[i] + delta[i];
                pred += delta[i] * (rhs[i] + mu * dd[i] * delta[i]);
            }
            clip_to(trial, n, fp->lo, fp->hi);
            Ft = fit_eval(fp, trial, Ht, gt, &chi2t, NULL);
            if (!isfinite(Ft)) Ft = INFINITY;
        }
        if (Ft < F) {
            double step = 0.0;
            for (int j = 0; j < m; ++j) {
                const double *tn = trial + 4 * j, *to = theta + 4 * j;
                double sa = fabs(tn[0]) > 1e-30 ? fabs(tn[0]) : 1e-30;
                double v;
                v = fabs(tn[0] - to[0]) / sa; if (v > step) step = v;
                v = fabs(tn[1] - to[1]) / tn[3]; if (v > step) step = v;
                v = fabs(tn[2] - to[2]) / tn[3]; if (v > step) step = v;
                v = fabs(tn[3] - to[3]) / tn[3]; if (v > step) step = v;
            }
            double rho = pred > 0.0 ? (F - Ft) / pred : 1.0;
            double t = 2.0 * rho - 1.0;
            double f = 1.0 - t * t * t;
            if (f < 1.0 / 3.0) f = 1.0 / 3.0;
            mu *= f;
            if (mu < 1e-12) mu = 1e-12;
            nu = 2.0;
            memcpy(theta, trial, sizeof(double) * (size_t)n);
            memcpy(Hs, Ht, sizeof(double) * (size_t)n * n);
            memcpy(g, gt, sizeof(double) * (size_t)n);
            F = Ft;
            chi2 = chi2t;
            if (step < tol) { res.converged = 1; break; }
        } else {
            mu *= nu;
            nu *= 2.0;
            if (mu > 1e8) { res.converged = 1; break; }
        }
    }
    res.F = F;
    res.chi2 = chi2;
    fit_eval(fp, theta, NULL, NULL, NULL, &res.npx);
    if (hess_out) memcpy(hess_out, Hs, sizeof(double) * (size_t)n * n);
    free(Hs); free(Ht); free(A);
    return res;
}

/* ------------------------------------------------------------------------ */
/* PSF main-lobe Gaussian (Sect. 3: the PSF is approximated by one Gaussian  */
/* with fixed alpha_b, omega_b).  Reading: centre at the PSF peak pixel;     */
/* the main lobe is the 4-connected region around the peak with             */
/* psf >= main_lobe_frac * peak; (alpha_b, omega_b) minimise the squared     */
/* error there (Gauss-Newton with Marquardt damping, to convergence).        */
/* ------------------------------------------------------------------------ */

int orc_psf_fit(const double *psf, int64_t Hp, int64_t Wp, double main_lobe_frac,
                double *alpha_b, double *omega_b, int64_t *n_lobe_px)
{
    int64_t n = Hp * Wp;
    if (Hp <= 0 || Wp <= 0) return ORC_ERR_ARG;
    int64_t pk = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(psf[i])) return ORC_ERR_NONFINITE;
        if (psf[i] > psf[pk]) pk = i;
    }
    double pv = psf[pk];
    if (!(pv > 0.0)) return ORC_ERR_PSF;
    double lim = main_lobe_frac * pv;
    unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *lobe = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!mark || !stack || !lobe) { free(mark); free(stack); free(lobe); return ORC_ERR_ARG; }
    int64_t sp = 0, nl = 0;
    stack[sp++] = pk; mark[pk] = 1;
    while (sp > 0) {
        int64_t i = stack[--sp];
        lobe[nl++] = i;
        int64_t r = i / Wp, c = i % Wp;
        int64_t nb[4] = {r > 0 ? i - Wp : -1, r < Hp - 1 ? i + Wp : -1,
                         c > 0 ? i - 1 : -1, c < Wp - 1 ? i + 1 : -1};
        for (int t = 0; t < 4; ++t) {
            int64_t j = nb[t];
            if (j >= 0 && !mark[j] && psf[j] >= lim) { mark[j] = 1; stack[sp++] = j; }
        }
    }
    free(stack); free(mark);
    int64_t pr = pk / Wp, pc = pk % Wp;
    double *q = (double *)malloc(sizeof(double) * (size_t)nl);
    double *v = (double *)malloc(sizeof(double) * (size_t)nl);
    for (int64_t t = 0; t < nl; ++t) {
        int64_t r = lobe[t] / Wp, c = lobe[t] % Wp;
        double dr = (double)(r - pr), dc = (double)(c - pc);
        q[t] = dr * dr + dc * dc;
        v[t] = psf[lobe[t]];
    }
    free(lobe);
    /* minimise sum_t (v_t - alpha exp(-q_t / (2 omega^2)))^2 over (alpha, omega) */
    double th[2] = {pv, sqrt((double)nl / (2.0 * ORC_PI * log(1.0 / main_lobe_frac)))};
    if (nl == 1) th[1] = 0.5;
    double mu = 1e-3;
    double Fcur = 0.0;
    for (int it = 0; it < 500; ++it) {
        double F = 0.0, h00 = 0, h01 = 0, h11 = 0, g0 = 0, g1 = 0;
        for (int64_t t = 0; t < nl; ++t) {
            double w2 = th[1] * th[1];
            double e = exp(-q[t] / (2.0 * w2));
            double G = th[0] * e;
            double j0 = e, j1 = G * q[t] / (w2 * th[1]);
            double r = v[t] - G;
            F += r * r; h00 += j0 * j0; h01 += j0 * j1; h11 += j1 * j1;
            g0 += j0 * r; g1 += j1 * r;
        }
        if (it == 0) Fcur = F;
        double gv[2] = {g0, g1};
        int accepted = 0, done = 0;
        while (mu <= 1e8) {
            double A[4] = {h00 * (1.0 + mu), h01, h01, h11 * (1.0 + mu)};
            double d[2];
            if (orc_cholesky_solve(2, A, gv, d) != 0) { mu *= 10.0; continue; }
            double t0 = th[0] + d[0], t1 = th[1] + d[1];
            if (!(t1 > 1e-3)) t1 = 1e-3;
            double Ft = 0.0;
            for (int64_t t = 0; t < nl; ++t) {
                double r = v[t] - t0 * exp(-q[t] / (2.0 * t1 * t1));
                Ft += r * r;
            }
            if (isfinite(Ft) && Ft < Fcur) {
                double step = fabs(t0 - th[0]) / fabs(t0) + fabs(t1 - th[1]) / t1;
                th[0] = t0; th[1] = t1; Fcur = Ft;
                mu = mu / 10.0 < 1e-12 ? 1e-12 : mu / 10.0;
                accepted = 1;
                done = step < 1e-14;
                break;
            }
            mu *= 10.0;
        }
        if (!accepted || done) break;
    }
    free(q); free(v);
    *alpha_b = th[0];
    *omega_b = th[1];
    if (n_lobe_px) *n_lobe_px = nl;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Active set (the paper names an active-set heuristic but defines it in     */
/* the 2004 paper, which is not available).  Reading: candidates are         */
/* existing components whose amplitude has the sign of the peak (zero       */
/* excluded) and whose centre lies inside the window of the simple start    */
/* (peak pixel, omega_b) whatever the new component's start value; they are */
/* taken most recent first up to K_max - 1 (with the sign bounds of the fit, */
/* no two members can cancel each other); a                                  */
/* candidate is skipped when it is too close to a member already taken (the */
/* new component first, at the simple start and, with a proposal, at the   */
/* proposal too): centres closer than                                        */
/* max(omega_b, min(s_j, s_m)), where two Gaussians of similar place and     */
/* width would make the joint fit degenerate.  Only FP64 products, sums,     */
/* min/max and compares of stored values: reproducible bit for bit.          */
/* ------------------------------------------------------------------------ */

static int too_close(double xj, double yj, double sj, double xm, double ym, double sm,
                     double omega_b)
{
    double ex = xj - xm, ey = yj - ym;
    double rs = sj < sm ? sj : sm;
    if (rs < omega_b) rs = omega_b;
    return ex * ex + ey * ey <= rs * rs;
}

static int select_active(const orc_state *st, const double *t0, const int64_t bnew[4],
                         const double *prop4, int32_t *chosen)
{
    int nch = 0;
    for (int64_t j = st->L - 1; j >= 0 && nch < st->max_active - 1; --j) {
        const orc_comp *cj = &st->comps[j];
        if (!(cj->a * t0[0] > 0.0)) continue;
        if (!(cj->y >= (double)bnew[0] && cj->y <= (double)bnew[1] &&
              cj->x >= (double)bnew[2] && cj->x <= (double)bnew[3])) continue;
        if (too_close(cj->x, cj->y, cj->s, t0[1], t0[2], t0[3], st->omega_b)) continue;
        /* a proposal start is a second place of the new component */
        if (prop4 && too_close(cj->x, cj->y, cj->s, prop4[1], prop4[2], prop4[3], st->omega_b))
            continue;
        int close = 0;
        for (int u = 0; u < nch && !close; ++u) {
            const orc_comp *cm = &st->comps[chosen[u]];
            close = too_close(cj->x, cj->y, cj->s, cm->x, cm->y, cm->s, st->omega_b);
        }
        if (close) continue;
        chosen[nch++] = (int32_t)j;
    }
    return nch;
}

/* ------------------------------------------------------------------------ */
/* One fit: select the active set around the start point (new component     */
/* first, then old members most recent first) and minimise F by LM.          */
/* Readings (bounds): every member keeps the sign its amplitude has at the   */
/* start of the fit; its centre stays inside its window at the start of the  */
/* fit (the component models the emission where it was found);              */
/* omega_b <= s <= s_max with s_max = max(omega_b, min(H, W) / 8) (Eq. 5     */
/* needs s >= omega_b; the upper bound keeps one component from spanning the */
/* field).                                                                   */
/* ------------------------------------------------------------------------ */

static double width_max(const orc_state *st)
{
    double smax = st->max_width > 0.0 ? st->max_width
                                      : (double)(st->H < st->W ? st->H : st->W) / 8.0;
    return smax > st->omega_b ? smax : st->omega_b;
}

static void set_bounds(fit_problem *fp, const double *theta)
{
    const orc_state *st = fp->st;
    for (int j = 0; j < fp->m; ++j) {
        int neg = theta[4 * j] < 0.0;
        fp->lo[4 * j + 0] = neg ? -INFINITY : 0.0;
        fp->hi[4 * j + 0] = neg ? 0.0 : INFINITY;
        int64_t w[4];
        comp_window(st, theta[4 * j + 1], theta[4 * j + 2], theta[4 * j + 3], w);
        fp->lo[4 * j + 1] = (double)w[2];    fp->hi[4 * j + 1] = (double)w[3];
        fp->lo[4 * j + 2] = (double)w[0];    fp->hi[4 * j + 2] = (double)w[1];
        fp->lo[4 * j + 3] = st->omega_b;
        fp->hi[4 * j + 3] = width_max(st);
    }
}

/* The active set depends on the peak and the component list only: it is
 * selected around the simple start `sel` (peak value, peak pixel, omega_b)
 * whatever the start `init4` of the new component.
 * With a proposal `prop4` (NULL for none) the new component has two starts,
 * the simple values init4 and the proposal; its centre bounds are the hull of
 * the two start windows, the objective is evaluated at both, and LM starts
 * from the lower one (the simple values on a tie).  *won = 1 when that is the
 * proposal. */
static int fit_from(const orc_state *st, const double *init4, const double *sel,
                    const double *prop4, int *won, orc_report *rep, double *theta,
                    lm_result *out, double *hess_out)
{
    double t0[4];
    memcpy(t0, init4, sizeof t0);
    int64_t wsel[4];
    comp_window(st, sel[1], sel[2], sel[3], wsel);
    int32_t chosen[ORC_MAX_ACTIVE];
    int nch = select_active(st, sel, wsel, prop4, chosen);
    fit_problem fp;
    memset(&fp, 0, sizeof fp);
    fp.st = st;
    fp.m = 1 + nch;
    fp.data = st->R;
    memcpy(theta, t0, sizeof t0);
    rep->members[0] = -1;
    for (int u = 0; u < nch; ++u) {
        const orc_comp *cj = &st->comps[chosen[u]];
        double *t = theta + 4 * (u + 1);
        t[0] = cj->a; t[1] = cj->x; t[2] = cj->y; t[3] = cj->s;
        rep->members[u + 1] = chosen[u];
        memcpy(fp.old + 4 * (u + 1), t, 4 * sizeof(double));
        comp_window(st, t[1], t[2], t[3], fp.wold[u + 1]);
    }
    rep->n_active = fp.m;
    set_bounds(&fp, theta);
    if (won) *won = 0;
    if (prop4) {
        int64_t wp[4];
        comp_window(st, prop4[1], prop4[2], prop4[3], wp);
        if ((double)wp[2] < fp.lo[1]) fp.lo[1] = (double)wp[2];
        if ((double)wp[3] > fp.hi[1]) fp.hi[1] = (double)wp[3];
        if ((double)wp[0] < fp.lo[2]) fp.lo[2] = (double)wp[0];
        if ((double)wp[1] > fp.hi[2]) fp.hi[2] = (double)wp[1];
        double alt[4 * ORC_MAX_ACTIVE];
        memcpy(alt, theta, sizeof(double) * 4 * (size_t)fp.m);
        memcpy(alt, prop4, 4 * sizeof(double));
        clip_to(alt, 4 * fp.m, fp.lo, fp.hi);
        clip_to(theta, 4 * fp.m, fp.lo, fp.hi);
        double Fs = fit_eval(&fp, theta, NULL, NULL, NULL, NULL);
        double Fp = fit_eval(&fp, alt, NULL, NULL, NULL, NULL);
        if (!isfinite(Fs)) Fs = INFINITY;
        if (Fp < Fs) {
            memcpy(theta, alt, sizeof(double) * 4 * (size_t)fp.m);
            if (won) *won = 1;
        }
    }
    memcpy(rep->theta0, theta, sizeof(double) * 4 * (size_t)fp.m);
    *out = lm_fit(&fp, theta, st->lm_max_iter, st->lm_mu0, st->lm_tol, hess_out);
    rep->omega_px = out->npx;
    return ORC_OK;
}

static void add_window(orc_state *st, double a, double x, double y, double s, double sign,
                       int64_t *touched)
{
    int64_t w[4];
    comp_window(st, x, y, s, w);
    for (int64_t r = w[0]; r <= w[1]; ++r)
        for (int64_t c = w[2]; c <= w[3]; ++c)
            st->R[r * st->W + c] += sign * gauss_at(a, x, y, s, r, c);
    *touched += (w[1] - w[0] + 1) * (w[3] - w[2] + 1);
}

static int step_impl(orc_state *st, const double *init, const double *start4, orc_report *rep,
                     double *hess_out)
{
    memset(rep, 0, sizeof *rep);
    int64_t n = st->H * st->W;
    /* The peak of the residual (Sect. 2 step 1; simple method of Sect. 3). */
    int64_t idx = orc_peak(st->R, n);
    double pv = st->R[idx];
    rep->idx = idx;
    rep->peak = pv;
    /* Stop criteria (Sect. 2 step 4): a noise threshold or an iteration count. */
    if (fabs(pv) < st->threshold) { rep->status = ORC_STOP_THRESHOLD; return rep->status; }
    if (st->k >= st->max_iter) { rep->status = ORC_STOP_MAXITER; return rep->status; }
    if (st->L >= st->cap) { rep->status = ORC_ERR_CAPACITY; return rep->status; }
    int64_t pr = idx / st->W, pc = idx % st->W;
    /* Simple initial values: the residual peak and the main-lobe width. */
    double plain[4] = {pv, (double)pc, (double)pr, st->omega_b};
    double theta[4 * ORC_MAX_ACTIVE];
    lm_result lmr;
    int used_fallback = 0, rc;
    if (start4) {
        /* Start values found elsewhere (the smoothing method of Sect. 2 step 1
         * and Sect. 3): the new component starts there, and the active set is
         * selected around that start, as it is around the simple start. */
        rc = fit_from(st, start4, start4, NULL, NULL, rep, theta, &lmr, hess_out);
        if (rc != ORC_OK) return rep->status = rc;
    } else if (init) {
        /* A proposal: width at least omega_b, centre within 16 px of the peak. */
        double p4[4] = {init[0], init[1], init[2], init[3]};
        if (!(p4[0] * pv > 0.0)) p4[0] = pv;     /* the peak's sign; also NaN */
        if (!(p4[1] >= (double)pc - 16.0)) p4[1] = (double)pc - 16.0;
        if (p4[1] > (double)pc + 16.0) p4[1] = (double)pc + 16.0;
        if (!(p4[2] >= (double)pr - 16.0)) p4[2] = (double)pr - 16.0;
        if (p4[2] > (double)pr + 16.0) p4[2] = (double)pr + 16.0;
        if (p4[1] < 0.0) p4[1] = 0.0;
        if (p4[1] > (double)(st->W - 1)) p4[1] = (double)(st->W - 1);
        if (p4[2] < 0.0) p4[2] = 0.0;
        if (p4[2] > (double)(st->H - 1)) p4[2] = (double)(st->H - 1);
        if (!(p4[3] >= st->omega_b)) p4[3] = st->omega_b;
        if (p4[3] > width_max(st)) p4[3] = width_max(st);
        int won = 0;
        rc = fit_from(st, plain, plain, p4, &won, rep, theta, &lmr, hess_out);
        if (rc != ORC_OK) return rep->status = rc;
        rep->start_from_proposal = won;
        if (won && (!lmr.converged || theta[0] == 0.0)) {
            /* The simple initial values are the fallback of a proposal that
             * failed: LM did not converge from it, or converged to a new
             * component of zero amplitude (a start that explains none of the
             * peak's emission; without the fallback such a fit can leave the
             * model unchanged and bring the same peak and the same proposal
             * back every iteration). */
            used_fallback = 1;
            int tr = lmr.trials;
            rc = fit_from(st, plain, plain, NULL, NULL, rep, theta, &lmr, hess_out);
            if (rc != ORC_OK) return rep->status = rc;
            lmr.trials += tr;
        }
    } else {
        rc = fit_from(st, plain, plain, NULL, NULL, rep, theta, &lmr, hess_out);
        if (rc != ORC_OK) return rep->status = rc;
    }
    int m = rep->n_active;
    memcpy(rep->theta, theta, sizeof(double) * 4 * (size_t)m);
    rep->lm_iters = lmr.trials;
    rep->converged = lmr.converged;
    rep->used_fallback = used_fallback;
    rep->chi2_init = lmr.chi2_0;
    rep->chi2_final = lmr.chi2;

    /* Commit and residual update (Sect. 2 step 3 with B = the Gaussian beam).
     * Reading of the loop gain (Sect. 3): every change the fit makes to the
     * model image is scaled by the gain.  The new component joins with gain
     * times its fitted amplitude, at its fitted centre and width; each old
     * member moves the fraction gain of the way from its stored parameters to
     * its refit, t_j <- t_j + gain (t*_j - t_j), and is added back on its old
     * window and subtracted on its new one.  A new component whose fitted
     * amplitude is zero (held on its sign bound: the old members explain the
     * peak) models no emission and is not added to the list. */
    int64_t touched = 0;
    const double g = st->gain;
    for (int j = 1; j < m; ++j) {
        orc_comp *cj = &st->comps[rep->members[j]];
        add_window(st, cj->a, cj->x, cj->y, cj->s, +1.0, &touched);
        const double *t = theta + 4 * j;
        cj->a = cj->a + g * (t[0] - cj->a);
        cj->x = cj->x + g * (t[1] - cj->x);
        cj->y = cj->y + g * (t[2] - cj->y);
        cj->s = cj->s + g * (t[3] - cj->s);
        cj->iter_updated = st->k;
        add_window(st, cj->a, cj->x, cj->y, cj->s, -1.0, &touched);
    }
    rep->added = theta[0] != 0.0;
    if (rep->added) {
        orc_comp *cn = &st->comps[st->L];
        cn->a = g * theta[0];
        cn->x = theta[1]; cn->y = theta[2]; cn->s = theta[3];
        cn->iter_added = st->k;
        cn->iter_updated = st->k;
        add_window(st, cn->a, cn->x, cn->y, cn->s, -1.0, &touched);
        st->L += 1;
    }
    st->k += 1;
    rep->update_px = touched;
    rep->status = lmr.converged ? ORC_OK : ORC_LM_NOT_CONVERGED;
    return rep->status;
}

int orc_step(orc_state *st, const double *init, orc_report *rep, double *hess_out)
{
    return step_impl(st, init, NULL, rep, hess_out);
}

int orc_step_start(orc_state *st, const double *start4, orc_report *rep, double *hess_out)
{
    if (!start4) return ORC_ERR_ARG;
    return step_impl(st, NULL, start4, rep, hess_out);
}

int orc_run(orc_state *st, int64_t n_iter, int64_t *done)
{
    orc_report rep;
    int rc = ORC_OK;
    int64_t i = 0;
    for (; i < n_iter; ++i) {
        rc = orc_step(st, NULL, &rep, NULL);
        if (rc != ORC_OK && rc != ORC_LM_NOT_CONVERGED) break;
    }
    if (done) *done = i;
    return rc;
}

void orc_residual_from_scratch(const orc_state *st, const double *dirty, double *out)
{
    int64_t n = st->H * st->W;
    memcpy(out, dirty, sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < st->L; ++j) {
        const orc_comp *cj = &st->comps[j];
        int64_t w[4];
        comp_window(st, cj->x, cj->y, cj->s, w);
        for (int64_t r = w[0]; r <= w[1]; ++r)
            for (int64_t c = w[2]; c <= w[3]; ++c)
                out[r * st->W + c] -= gauss_at(cj->a, cj->x, cj->y, cj->s, r, c);
    }
}

int orc_fit_gaussians(const double *data, int64_t H, int64_t W, int m, double *theta,
                      double omega_b, double max_width, double window_sigmas, int lm_max_iter,
                      double mu0, double tol, int32_t *converged, double *chi2)
{
    if (m < 1 || m > ORC_MAX_ACTIVE) return -1;
    orc_state st;
    memset(&st, 0, sizeof st);
    orc_default_config(&st);
    st.H = H; st.W = W;
    st.window_sigmas = window_sigmas;
    st.omega_b = omega_b;
    st.max_width = max_width;
    fit_problem fp;
    memset(&fp, 0, sizeof fp);
    fp.st = &st;
    fp.m = m;
    fp.data = data;
    /* no old members to add back: every stored window is empty */
    for (int j = 0; j < m; ++j) {
        fp.wold[j][0] = 0; fp.wold[j][1] = -1; fp.wold[j][2] = 0; fp.wold[j][3] = -1;
    }
    set_bounds(&fp, theta);
    lm_result r = lm_fit(&fp, theta, lm_max_iter, mu0, tol, NULL);
    if (converged) *converged = r.converged;
    if (chi2) *chi2 = r.chi2;
    return r.trials;
}
