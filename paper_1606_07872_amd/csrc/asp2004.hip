// The Asp-Clean2004 iteration, the comparison path of the paper (Sect. 2,
// steps 1-4, with the objective of Eq. 3 and the cost count that follows it;
// Table 3).  The new component is fitted in the sky plane, theta = (F, x, y,
// v = omega^2), by Levenberg-Marquardt against
//     chi^2(theta) = || R - B (*) g(theta) ||^2   over the whole image,
// with the true PSF B convolved in every evaluation -- the convolution the
// 2016 method removes.  g is rendered as the exact-PSF refresh renders the
// model (a sampled Gaussian of flux F for omega >= 1 px; below, per axis three
// Gauss-Hermite nodes spread by Lanczos-3 and normalised), and the Jacobian
// columns are B (*) dg/dtheta_k with the derivatives of that rendering.  The
// rendering is even in omega; in v = omega^2 its derivative stays finite and
// in general non-zero at a point source (the limit is half the profile's
// second derivative), so a fit can leave the bound v = 0.
//
// An evaluation: the unit-flux image and its three derivative images are
// rendered into four zero-padded FP64 grids, transformed by one batched
// hipFFT D2Z, multiplied by the PSF's spectrum, transformed back by one
// batched Z2D; one pass over the image forms the 4 x 4 Gram matrix, J^T r,
// F = sum m (m - 2 R) and chi^2 in FP64, as per-work-group partial sums; one
// work-group adds them in a fixed order and takes the LM decision.  The LM
// rules are those of the 2016 fit (damped normal equations with a bound
// guard, gain-ratio damping, step test, stall at mu > 1e8).
#include <hipfft/hipfft.h>

#include "asp_device.h"

namespace asp {
namespace {

constexpr int kT = 256;
constexpr int kTaps = 12;
constexpr double kPi = 3.14159265358979323846;

__device__ inline bool live(const A4Args &a) { return a.st->stop == 0 && a.s->done == 0; }
__device__ inline bool finished(const A4Args &a) { return a.st->stop == 0 && a.s->done == 1; }

__device__ inline double sinc(double t)
{
    return t == 0.0 ? 1.0 : sinpi(t) / (kPi * t);
}

// d/dt sinc(t); a series near 0, where the closed form cancels.
__device__ inline double dsinc(double t)
{
    if (fabs(t) < 1e-3) {
        const double p2 = kPi * kPi;
        return -p2 * t / 3.0 + p2 * p2 * t * t * t / 30.0;
    }
    return (cospi(t) - sinc(t)) / t;
}

// d^2/dt^2 sinc(t)
__device__ inline double d2sinc(double t)
{
    const double p2 = kPi * kPi;
    if (fabs(t) < 1e-3) return -p2 / 3.0 + p2 * p2 * t * t / 10.0;
    return -p2 * sinc(t) - 2.0 * dsinc(t) / t;
}

__device__ inline double lanczos3(double t)
{
    return fabs(t) < 3.0 ? sinc(t) * sinc(t / 3.0) : 0.0;
}

__device__ inline double lanczos3_deriv(double t)
{
    return fabs(t) < 3.0 ? dsinc(t) * sinc(t / 3.0) + sinc(t) * dsinc(t / 3.0) / 3.0 : 0.0;
}

__device__ inline double lanczos3_deriv2(double t)
{
    if (!(fabs(t) < 3.0)) return 0.0;
    const double u = t / 3.0;
    return d2sinc(t) * sinc(u) + 2.0 * dsinc(t) * dsinc(u) / 3.0 + sinc(t) * d2sinc(u) / 9.0;
}

constexpr double kSmallWidth = 1e-4;   // px: below, dg/dv takes its limit at omega = 0

__global__ __launch_bounds__(kT) void k_a4_zero(A4Args a, int images, int final_only)
{
    if (final_only ? !finished(a) : !live(a)) return;
    const int64_t n = (int64_t)images * a.Py * a.Px;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        a.grid[i] = 0.0;
}

// The unit-flux component at (x, y) with squared width v and, unless final,
// its derivative images in x, y and v, into the grids (the image occupies
// rows 0..H-1, columns 0..W-1 of each).
__global__ __launch_bounds__(kT) void k_a4_render(A4Args a, int final_img)
{
    if (final_img ? !finished(a) : !live(a)) return;
    const double *th = final_img ? a.s->theta : a.s->te;
    const double x = th[1], y = th[2], v = th[3], om = sqrt(v);
    const int64_t plane = a.Py * a.Px;
    if (om >= 1.0) {
        const int h = halfwidth(om, a.window_sigmas);
        const int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
        const int64_t r0 = cy - h < 0 ? 0 : cy - h, r1 = cy + h > a.H - 1 ? a.H - 1 : cy + h;
        const int64_t c0 = cx - h < 0 ? 0 : cx - h, c1 = cx + h > a.W - 1 ? a.W - 1 : cx + h;
        if (r0 > r1 || c0 > c1) return;
        const int64_t wc = c1 - c0 + 1, n = (r1 - r0 + 1) * wc;
        const double norm = 1.0 / (2.0 * kPi * v);
        for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kT) {
            const int64_t r = r0 + i / wc, c = c0 + i % wc;
            const double dx = (double)c - x, dy = (double)r - y;
            const double q = dx * dx + dy * dy;
            const double e = exp(-q / (2.0 * v)) * norm;
            const int64_t o = r * a.Px + c;
            a.grid[o] = e;
            if (final_img) continue;
            a.grid[plane + o] = e * dx / v;
            a.grid[2 * plane + o] = e * dy / v;
            a.grid[3 * plane + o] = e * (q / (2.0 * v * v) - 1.0 / v);
        }
        return;
    }
    // narrow: one work-group, the 12 x 12 taps
    if (blockIdx.x != 0) return;
    __shared__ double u[2][kTaps], ud[2][kTaps], uw[2][kTaps];
    __shared__ double w[2][kTaps], wd[2][kTaps], ww[2][kTaps];
    const int t = threadIdx.x;
    const double d1 = 1.7320508075688772 * om;            // sqrt(3) omega
    const int64_t b0[2] = {(int64_t)floor(x) - 5, (int64_t)floor(y) - 5};
    if (t < 2 * kTaps) {
        const int ax = t / kTaps, k = t % kTaps;
        const double ctr = ax == 0 ? x : y;
        const double tt = (double)(b0[ax] + k) - ctr;
        const double tm = tt - d1, tp = tt + d1;
        u[ax][k] = (2.0 / 3.0) * lanczos3(tt) + (1.0 / 6.0) * lanczos3(tm) + (1.0 / 6.0) * lanczos3(tp);
        const double l0 = lanczos3_deriv(tt), lm = lanczos3_deriv(tm), lp = lanczos3_deriv(tp);
        ud[ax][k] = -((2.0 / 3.0) * l0 + (1.0 / 6.0) * lm + (1.0 / 6.0) * lp);
        // d/dv of p L(t - d omega) is -p d L'(...) / (2 omega), nodes at +-sqrt(3);
        // as omega -> 0 the sum tends to sum p d^2 L''(t) / 2 = L''(t) / 2
        uw[ax][k] = om >= kSmallWidth
            ? -((1.0 / 6.0) * 1.7320508075688772 * lm - (1.0 / 6.0) * 1.7320508075688772 * lp) /
                  (2.0 * om)
            : 0.5 * lanczos3_deriv2(tt);
    }
    __syncthreads();
    if (t < 2) {
        double S = 0.0, Sd = 0.0, Sw = 0.0;
        for (int k = 0; k < kTaps; ++k) { S += u[t][k]; Sd += ud[t][k]; Sw += uw[t][k]; }
        for (int k = 0; k < kTaps; ++k) {
            const double wk = u[t][k] / S;
            w[t][k] = wk;
            wd[t][k] = (ud[t][k] - wk * Sd) / S;
            ww[t][k] = (uw[t][k] - wk * Sw) / S;
        }
    }
    __syncthreads();
    if (t < kTaps * kTaps) {
        const int i = t / kTaps, j = t % kTaps;
        const int64_t r = b0[1] + i, c = b0[0] + j;
        if (r < 0 || r >= a.H || c < 0 || c >= a.W) return;
        const int64_t o = r * a.Px + c;
        a.grid[o] = w[1][i] * w[0][j];
        if (final_img) return;
        a.grid[plane + o] = w[1][i] * wd[0][j];
        a.grid[2 * plane + o] = wd[1][i] * w[0][j];
        a.grid[3 * plane + o] = ww[1][i] * w[0][j] + w[1][i] * ww[0][j];
    }
}

// The spectra times the PSF's, with the 1 / (Py Px) of the inverse.
__global__ __launch_bounds__(kT) void k_a4_mul(A4Args a, int images, int final_only)
{
    if (final_only ? !finished(a) : !live(a)) return;
    const int64_t m = a.Py * (a.Px / 2 + 1);
    const double scale = 1.0 / ((double)a.Py * (double)a.Px);
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) {
        const double2 b = a.pspec[i];
        for (int img = 0; img < images; ++img) {
            const double2 v = a.spec[img * m + i];
            a.spec[img * m + i] =
                make_double2((v.x * b.x - v.y * b.y) * scale, (v.x * b.y + v.y * b.x) * scale);
        }
    }
}

// Per work-group partial sums over the image of the Gram matrix of
// J = (B(*)g, F B(*)g_x, F B(*)g_y, F B(*)g_v), of J^T r with r = R - F B(*)g,
// of m (m - 2 R) and of r^2.  Pixel (r, c) of the convolution sits at
// (r + ci, c + cj) of the full linear convolution.  Work-group b takes rows
// b, b + nblk, ...; the sums are reduced in a fixed order (wave butterflies,
// then the waves in order).
__global__ __launch_bounds__(kT) void k_a4_gram(A4Args a)
{
    if (!live(a)) return;
    __shared__ double red[kT / 64][kA4Sums];
    const double F = a.s->te[0];
    const int64_t plane = a.Py * a.Px;
    double acc[kA4Sums];
#pragma unroll
    for (int k = 0; k < kA4Sums; ++k) acc[k] = 0.0;
    for (int64_t r = blockIdx.x; r < a.H; r += gridDim.x) {
        const double *g0 = a.grid + (r + a.ci) * a.Px + a.cj;
        const float *Rr = a.R + r * a.W;
        for (int64_t c = threadIdx.x; c < a.W; c += kT) {
            const double v0 = g0[c];
            const double J[4] = {v0, F * g0[plane + c], F * g0[2 * plane + c], F * g0[3 * plane + c]};
            const double D = (double)Rr[c];
            const double m = F * v0, res = D - m;
            int e = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = p; q < 4; ++q) acc[e++] += J[p] * J[q];
#pragma unroll
            for (int p = 0; p < 4; ++p) acc[10 + p] += J[p] * res;
            acc[14] += m * (m - 2.0 * D);
            acc[15] += res * res;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kA4Sums; ++k) {
        double v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kA4Sums) {
        double v = 0.0;
        for (int q = 0; q < kT / 64; ++q) v += red[q][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * kA4Sums + threadIdx.x] = v;
    }
}

__device__ inline double clampd(double v, double lo, double hi)
{
    if (!(v >= lo)) v = lo;
    if (v > hi) v = hi;
    return v;
}

// Cholesky solve of the 4 x 4 system A x = b (row-major); false if A is not
// positive definite.
__device__ bool chol4(const double *A, const double *b, double *x)
{
    double L[16] = {0.0};
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k <= i; ++k) {
            double s = A[i * 4 + k];
            for (int j = 0; j < k; ++j) s -= L[i * 4 + j] * L[k * 4 + j];
            if (i == k) {
                if (!(s > 0.0)) return false;
                L[i * 4 + i] = sqrt(s);
            } else {
                L[i * 4 + k] = s / L[k * 4 + k];
            }
        }
    double z[4];
    for (int i = 0; i < 4; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= L[i * 4 + j] * z[j];
        z[i] = s / L[i * 4 + i];
    }
    for (int i = 3; i >= 0; --i) {
        double s = z[i];
        for (int j = i + 1; j < 4; ++j) s -= L[j * 4 + i] * x[j];
        x[i] = s / L[i * 4 + i];
    }
    return true;
}

// Propose the next trial from (theta, Hs, g, mu): on success s->te holds it
// and phase = 1; a system that is not positive definite counts as a
// rejected trial.  Ends the fit on the budget or a stall.
__device__ void propose(const A4Args &a, A4State *s)
{
    for (;;) {
        if (s->trials >= a.budget) { s->done = 1; return; }
        double dmax = 0.0;
        for (int i = 0; i < 4; ++i) dmax = s->Hs[i * 5] > dmax ? s->Hs[i * 5] : dmax;
        double A[16], rhs[4], delta[4];
        for (int i = 0; i < 16; ++i) A[i] = s->Hs[i];
        for (int i = 0; i < 4; ++i) {
            rhs[i] = s->g[i];
            double d = s->Hs[i * 5];
            if (d < 1e-12 * dmax) d = 1e-12 * dmax;
            s->dd[i] = d;
            A[i * 5] += s->mu * d;
        }
        for (int i = 0; i < 4; ++i) {
            if ((s->theta[i] <= s->lo[i] && s->g[i] <= 0.0) ||
                (s->theta[i] >= s->hi[i] && s->g[i] >= 0.0)) {
                for (int k = 0; k < 4; ++k) { A[i * 4 + k] = 0.0; A[k * 4 + i] = 0.0; }
                A[i * 5] = 1.0;
                rhs[i] = 0.0;
            }
        }
        s->trials += 1;
        if (chol4(A, rhs, delta)) {
            double pred = 0.0;
            for (int i = 0; i < 4; ++i) {
                pred += delta[i] * (rhs[i] + s->mu * s->dd[i] * delta[i]);
                s->te[i] = clampd(s->theta[i] + delta[i], s->lo[i], s->hi[i]);
            }
            s->pred = pred;
            s->phase = 1;
            return;
        }
        s->mu *= s->nu;
        s->nu *= 2.0;
        if (s->mu > 1e8) { s->converged = 1; s->done = 1; return; }
    }
}

// Sum the partial rows in a fixed order, then the LM decision on the point
// just evaluated and the next trial.
__global__ __launch_bounds__(kT) void k_a4_lm(A4Args a)
{
    if (!live(a)) return;
    // thread t adds column t % 16 of rows t / 16, t / 16 + 16, ...; then the
    // 16 row groups are added in order
    __shared__ double grp[kT / kA4Sums][kA4Sums];
    __shared__ double tot[kA4Sums];
    const int t = threadIdx.x;
    {
        const int k = t % kA4Sums, g0 = t / kA4Sums;
        double v = 0.0;
        for (int b = g0; b < a.nblk; b += kT / kA4Sums) v += a.partials[(int64_t)b * kA4Sums + k];
        grp[g0][k] = v;
    }
    __syncthreads();
    if (t < kA4Sums) {
        double v = 0.0;
        for (int q = 0; q < kT / kA4Sums; ++q) v += grp[q][t];
        tot[t] = v;
    }
    __syncthreads();
    if (t != 0) return;
    A4State *s = a.s;
    s->evals += 1;
    double Hn[16], gn[4];
    int e = 0;
    for (int p = 0; p < 4; ++p)
        for (int q = p; q < 4; ++q) { Hn[p * 4 + q] = tot[e]; Hn[q * 4 + p] = tot[e]; ++e; }
    for (int p = 0; p < 4; ++p) gn[p] = tot[10 + p];
    const double obj = tot[14], chi2 = tot[15];
    if (s->phase == 0) {
        s->F = obj; s->F0 = obj; s->chi2 = chi2; s->chi2_init = chi2;
        for (int i = 0; i < 16; ++i) s->Hs[i] = Hn[i];
        for (int i = 0; i < 4; ++i) s->g[i] = gn[i];
    } else {
        const double Ft = isfinite(obj) ? obj : INFINITY;
        if (Ft < s->F) {
            const double *tn = s->te, *to = s->theta;
            const double s2 = tn[3] + a.st->omega_b * a.st->omega_b, st = sqrt(s2);
            const double sa = fabs(tn[0]) > 1e-30 ? fabs(tn[0]) : 1e-30;
            double step = fabs(tn[0] - to[0]) / sa;
            for (int i = 1; i < 3; ++i) {
                const double v = fabs(tn[i] - to[i]) / st;
                step = v > step ? v : step;
            }
            const double sv = fabs(tn[3] - to[3]) / s2;
            step = sv > step ? sv : step;
            const double rho = s->pred > 0.0 ? (s->F - Ft) / s->pred : 1.0;
            const double u = 2.0 * rho - 1.0;
            double f = 1.0 - u * u * u;
            if (f < 1.0 / 3.0) f = 1.0 / 3.0;
            s->mu *= f;
            if (s->mu < 1e-12) s->mu = 1e-12;
            s->nu = 2.0;
            for (int i = 0; i < 4; ++i) s->theta[i] = s->te[i];
            for (int i = 0; i < 16; ++i) s->Hs[i] = Hn[i];
            for (int i = 0; i < 4; ++i) s->g[i] = gn[i];
            s->F = Ft;
            s->chi2 = chi2;
            if (step < a.tol) { s->converged = 1; s->done = 1; return; }
        } else {
            s->mu *= s->nu;
            s->nu *= 2.0;
            if (s->mu > 1e8) { s->converged = 1; s->done = 1; return; }
        }
    }
    propose(a, s);
}

// After the peak and the smoothing pick: the peak slots cleared, the capacity
// check, the start in the sky plane (Eq. 5 from the smoothing start,
// v_0 = max(s^2 - omega_b^2, 0)) and the bounds.
__global__ void k_a4_begin(A4Args a)
{
    // the peak key has been decoded: clear its slots for the next search
    for (int t = threadIdx.x; t < kPeakSlots; t += blockDim.x)
        __hip_atomic_store(&a.st->peak_keys[t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x != 0) return;
    DevState *st = a.st;
    A4State *s = a.s;
    s->done = 1;
    s->phase = 0;
    s->trials = 0;
    s->converged = 0;
    s->evals = 0;
    if (st->stop) return;
    if (st->L >= a.cap) { st->stop = ASP_ERR_CAPACITY; return; }
    if (!st->smooth_ready) { st->stop = ASP_ERR_STATE; return; }
    const double ab = st->alpha_b, wb = st->omega_b;
    const double ac = st->smooth_start[0], x0 = st->smooth_start[1], y0 = st->smooth_start[2];
    const double sg = st->smooth_start[3];
    const double w2 = __dsub_rn(__dmul_rn(sg, sg), __dmul_rn(wb, wb));
    const double v0 = w2 > 0.0 ? w2 : 0.0;
    const double F0 = __ddiv_rn(__dmul_rn(__dmul_rn(ac, sg), sg), __dmul_rn(__dmul_rn(ab, wb), wb));
    const double s0 = sqrt(__dadd_rn(v0, __dmul_rn(wb, wb)));
    int32_t box[4];
    make_window(x0, y0, halfwidth(s0, a.window_sigmas), a.H, a.W, box);
    const bool neg = F0 < 0.0;
    const double m2 = __dsub_rn(__dmul_rn(a.s_max, a.s_max), __dmul_rn(wb, wb));
    s->lo[0] = neg ? -INFINITY : 0.0;
    s->hi[0] = neg ? 0.0 : INFINITY;
    s->lo[1] = (double)box[2]; s->hi[1] = (double)box[3];
    s->lo[2] = (double)box[0]; s->hi[2] = (double)box[1];
    s->lo[3] = 0.0;
    s->hi[3] = m2 > 0.0 ? m2 : 0.0;
    const double t0[4] = {F0, x0, y0, v0};
    for (int i = 0; i < 4; ++i) {
        const double v = clampd(t0[i], s->lo[i], s->hi[i]);
        s->theta0[i] = v;
        s->theta[i] = v;
        s->te[i] = v;
    }
    s->mu = a.mu0;
    s->nu = 2.0;
    s->pred = 0.0;
    s->done = 0;
}

// R -= (gain F) B(*)g(theta), rounded to FP32.
__global__ __launch_bounds__(kT) void k_a4_update(A4Args a)
{
    if (!finished(a)) return;
    const double gF = a.gain * a.s->theta[0];
    for (int64_t r = blockIdx.x; r < a.H; r += gridDim.x) {
        const double *g0 = a.grid + (r + a.ci) * a.Px + a.cj;
        float *Rr = a.R + r * a.W;
        for (int64_t c = threadIdx.x; c < a.W; c += kT) Rr[c] = (float)((double)Rr[c] - gF * g0[c]);
    }
}

// The new component, kept as the convolved-space Gaussian whose Eqs. 5-6
// deconvolution is (gain F, omega = sqrt(v)), and the iteration's report.
__global__ void k_a4_append(A4Args a)
{
    if (threadIdx.x != 0 || !finished(a)) return;
    DevState *st = a.st;
    const A4State *s = a.s;
    const double ab = st->alpha_b, wb = st->omega_b;
    const double Fc = a.gain * s->theta[0], om = sqrt(s->theta[3]);
    const double sc = sqrt(__dadd_rn(__dmul_rn(om, om), __dmul_rn(wb, wb)));
    const int64_t L = st->L;
    a.ca[L] = __ddiv_rn(__dmul_rn(__dmul_rn(__dmul_rn(Fc, ab), wb), wb), __dmul_rn(sc, sc));
    a.cx[L] = s->theta[1];
    a.cy[L] = s->theta[2];
    a.cs[L] = sc;
    a.c_added[L] = st->k;
    a.c_updated[L] = st->k;
    st->n_active = 1;
    st->members[0] = -1;
    st->lm_iters = s->trials;
    st->converged = s->converged;
    st->used_fallback = 0;
    st->init_source = 3;
    st->start_prop = 0;
    for (int i = 0; i < 4; ++i) {
        st->init[i] = st->smooth_start[i];
        st->theta0[i] = s->theta0[i];
        st->theta[i] = s->theta[i];
    }
    st->chi2_init = s->chi2_init;
    st->chi2_final = s->chi2;
    st->fit_px = a.H * a.W;
    st->sum_trials += (unsigned long long)s->trials;
    st->not_converged += s->converged ? 0ull : 1ull;
    st->sum_smoothed += 1ull;
    st->sum_eval_px += (unsigned long long)s->evals * (unsigned long long)(a.H * a.W);
    st->smooth_ready = 0;
    st->L = L + 1;
    st->k = st->k + 1;
}

hipError_t fft_status(hipfftResult r)
{
    return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown;
}

}  // namespace

hipError_t a4_begin(const A4Args &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_begin, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t a4_trial(const A4Args &a, void *plan_fwd4, void *plan_inv4, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_zero, dim3(2048), dim3(kT), 0, s, a, 4, 0);
    hipLaunchKernelGGL(k_a4_render, dim3(1024), dim3(kT), 0, s, a, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecD2Z(*(hipfftHandle *)plan_fwd4, a.grid, (hipfftDoubleComplex *)a.spec));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_mul, dim3(2048), dim3(kT), 0, s, a, 4, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecZ2D(*(hipfftHandle *)plan_inv4, (hipfftDoubleComplex *)a.spec, a.grid));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_gram, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_lm, dim3(1), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t a4_commit(const A4Args &a, void *plan_fwd, void *plan_inv, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_zero, dim3(2048), dim3(kT), 0, s, a, 1, 1);
    hipLaunchKernelGGL(k_a4_render, dim3(1024), dim3(kT), 0, s, a, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecD2Z(*(hipfftHandle *)plan_fwd, a.grid, (hipfftDoubleComplex *)a.spec));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_mul, dim3(2048), dim3(kT), 0, s, a, 1, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecZ2D(*(hipfftHandle *)plan_inv, (hipfftDoubleComplex *)a.spec, a.grid));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_update, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_append, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace asp
