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
// Every image the rendering makes is a sum of outer products of per-axis
// factors (row factor a, column factor b): g = a0 (x) b0, dg/dx = a0 (x) b1,
// dg/dy = a1 (x) b0, dg/dv = a2 (x) b0 + a0 (x) b2.  For the sampled Gaussian
// e = exp(-dy^2/2v) exp(-dx^2/2v) / (2 pi v), and q/(2v^2) - 1/v splits into a
// row and a column term; for the narrow rendering the factors are the
// per-axis taps.  k_a4_taps computes them at the point under evaluation.
//
// An evaluation by FFT: the spectra of the four images are products of the
// factors' 1-D DFTs (k_a4_dft), so no grid is rendered or transformed
// forward; times the PSF's spectrum (k_a4_mulsep), transformed back by one
// batched hipFFT Z2D into four padded FP64 grids; one pass over the image
// forms the 4 x 4 Gram matrix, J^T r, F = sum m (m - 2 R) and chi^2 in FP64,
// as per-work-group partial sums (k_a4_gram); one work-group adds them in a
// fixed order and takes the LM decision (k_a4_lm).  The LM rules are those of
// the 2016 fit (damped normal equations with a bound guard, gain-ratio
// damping, step test, stall at mu > 1e8).  The same evaluation, and the
// update, can instead convolve directly, as two 1-D passes over the PSF
// (k_a4_xpass / k_a4_ypass); the host picks the cheaper per evaluation.
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

// One tap of one axis of the narrow rendering before normalisation: the
// profile u, its derivative in the centre ud and in v = omega^2 uw, at offset
// tt = tap - centre, from three Gauss-Hermite nodes (weights 2/3, 1/6, 1/6 at
// 0, -+sqrt(3) omega) spread by Lanczos-3.
__device__ inline void narrow_tap(double tt, double om, double *u, double *ud, double *uw)
{
    const double d1 = 1.7320508075688772 * om;            // sqrt(3) omega
    const double tm = tt - d1, tp = tt + d1;
    *u = (2.0 / 3.0) * lanczos3(tt) + (1.0 / 6.0) * lanczos3(tm) + (1.0 / 6.0) * lanczos3(tp);
    const double l0 = lanczos3_deriv(tt), lm = lanczos3_deriv(tm), lp = lanczos3_deriv(tp);
    *ud = -((2.0 / 3.0) * l0 + (1.0 / 6.0) * lm + (1.0 / 6.0) * lp);
    // d/dv of p L(t - d omega) is -p d L'(...) / (2 omega), nodes at +-sqrt(3);
    // as omega -> 0 the sum tends to sum p d^2 L''(t) / 2 = L''(t) / 2
    *uw = om >= kSmallWidth
        ? -((1.0 / 6.0) * 1.7320508075688772 * lm - (1.0 / 6.0) * 1.7320508075688772 * lp) /
              (2.0 * om)
        : 0.5 * lanczos3_deriv2(tt);
}

// The spectra of the grids by separability.  The image occupies rows
// 0..H-1 and columns 0..W-1 of a Py x Px grid; a grid a (x) b holding row
// factor a on rows R0.. and column factor b on columns C0.. has the D2Z
// half spectrum A[ky] Bc[kx] with the 1-D DFTs
//     A[ky] = sum_i a[i] exp(-2 pi i ky (R0 + i) / Py),  ky < Py,
//     Bc[kx] = sum_j b[j] exp(-2 pi i kx (C0 + j) / Px), kx <= Px / 2,
// so the forward transforms of the rendering are replaced by these sums.
// Each phase is reduced to (-Py/2, Py/2] in integers first, so conjugate
// frequencies get exactly conjugate values.
__device__ inline double2 dft_term(int64_t k, int64_t n, int64_t P)
{
    int64_t m = (k * n) % P;
    if (m < 0) m += P;
    if (2 * m > P) m -= P;
    double sn, cs;
    sincospi(-2.0 * (double)m / (double)P, &sn, &cs);
    return make_double2(cs, sn);
}

// The 1-D DFTs of the NF row and column factors in a.taps: rows into fac[f Py
// + ky], columns into fac[3 Py + f (Px/2 + 1) + kx].  One wave per frequency,
// the taps spread over its lanes and summed by a butterfly.
template <int NF>
__global__ __launch_bounds__(kT) void k_a4_dft(A4Args a)
{
    if (NF == 1 ? !finished(a) : !live(a)) return;
    const int64_t C0 = a.tapi[0], nc = a.tapi[1], R0 = a.tapi[2], nr = a.tapi[3];
    const int64_t hx = a.Px / 2 + 1, n = a.Py + hx;
    const double *bx = a.taps, *ay = a.taps + 3 * a.W;
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (kT / 64);
    for (int64_t q = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6); q < n; q += nwaves) {
        const bool row = q < a.Py;
        const int64_t k = row ? q : q - a.Py, P = row ? a.Py : a.Px;
        const int64_t cnt = row ? nr : nc, first = row ? R0 : C0, stride = row ? a.H : a.W;
        const double *fac = row ? ay : bx;
        double re[NF], im[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) { re[f] = 0.0; im[f] = 0.0; }
        for (int64_t j = lane; j < cnt; j += 64) {
            const double2 e = dft_term(k, first + j, P);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double v = fac[f * stride + j];
                re[f] += v * e.x;
                im[f] += v * e.y;
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
            for (int off = 32; off > 0; off >>= 1) {
                re[f] += __shfl_xor(re[f], off, 64);
                im[f] += __shfl_xor(im[f], off, 64);
            }
        if (lane == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int64_t o = row ? f * a.Py + k : 3 * a.Py + f * hx + k;
                a.fac[o] = make_double2(re[f], im[f]);
            }
        }
    }
}

__device__ inline double2 cmul(double2 u, double2 v)
{
    return make_double2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
}

// The spectra of g (and, for an evaluation, of dg/dx, dg/dy, dg/dv) from the
// factor DFTs, times the PSF's spectrum and the 1 / (Py Px) of the inverse:
// g = a0 (x) b0, dg/dx = a0 (x) b1, dg/dy = a1 (x) b0, dg/dv = a2 (x) b0 +
// a0 (x) b2.  An empty footprint gives zero spectra.
template <int NI>
__global__ __launch_bounds__(kT) void k_a4_mulsep(A4Args a)
{
    if (NI == 1 ? !finished(a) : !live(a)) return;
    const int64_t hx = a.Px / 2 + 1, m = a.Py * hx;
    const bool empty = a.tapi[1] == 0 || a.tapi[3] == 0;
    const double scale = empty ? 0.0 : 1.0 / ((double)a.Py * (double)a.Px);
    const double2 *A = a.fac, *B = a.fac + 3 * a.Py;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < m; i += (int64_t)gridDim.x * kT) {
        const int64_t ky = i / hx, kx = i - ky * hx;
        double2 b = a.pspec[i];
        b.x *= scale; b.y *= scale;
        const double2 a0 = A[ky], b0 = B[kx];
        a.spec[i] = cmul(cmul(a0, b0), b);
        if (NI == 1) continue;
        const double2 a1 = A[a.Py + ky], a2 = A[2 * a.Py + ky];
        const double2 b1 = B[hx + kx], b2 = B[2 * hx + kx];
        const double2 sv0 = cmul(a2, b0), sv1 = cmul(a0, b2);
        a.spec[m + i] = cmul(cmul(a0, b1), b);
        a.spec[2 * m + i] = cmul(cmul(a1, b0), b);
        a.spec[3 * m + i] = cmul(make_double2(sv0.x + sv1.x, sv0.y + sv1.y), b);
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

// ---------------------------------------------------------------------------
// The same evaluation without FFTs: B (*) (a (x) b) is a pass along the rows
// of B with b, then a pass along the columns with a; linear in the taps,
// exact up to rounding, and for narrow or moderately wide components cheaper
// than the padded transforms.
//
//   k_a4_taps   the factors at the point under evaluation, clipped to the
//               image: b_f on columns C0..C0+nc-1, a_f on rows R0..R0+nr-1;
//   k_a4_xpass  T_f(y, c) = sum_j b_f[j] B(y + yoff, c + cj - C0 - j) for the
//               H + nr - 1 rows of B any output row reaches (yoff = ci - R0 -
//               nr + 1), into the first planes of the grids;
//   k_a4_ypass  out(r, c) = sum_i a[i] T(r + nr - 1 - i, c), then the sums of
//               k_a4_gram (or the update of k_a4_update) at every pixel.
// ---------------------------------------------------------------------------

// The factors at s->te (s->theta for the update) into a.taps (b_f at f W,
// a_f at 3 W + f H) and a.tapi = {C0, nc, R0, nr}; an empty footprint gives
// nc = nr = 0.  With check_cap (the direct convolution) it ends the fit with
// ASP_ERR_STATE if the row pass would not fit the grids (the host never asks
// for that).
__global__ __launch_bounds__(kT) void k_a4_taps(A4Args a, int final_img, int check_cap)
{
    if (final_img ? !finished(a) : !live(a)) return;
    const double *th = final_img ? a.s->theta : a.s->te;
    const double x = th[1], y = th[2], v = th[3], om = sqrt(v);
    double *bx = a.taps, *ay = a.taps + 3 * a.W;
    const int t = threadIdx.x;
    int64_t C0, nc, R0, nr;
    if (om >= 1.0) {
        const int h = halfwidth(om, a.window_sigmas);
        const int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
        const int64_t r0 = cy - h < 0 ? 0 : cy - h, r1 = cy + h > a.H - 1 ? a.H - 1 : cy + h;
        const int64_t c0 = cx - h < 0 ? 0 : cx - h, c1 = cx + h > a.W - 1 ? a.W - 1 : cx + h;
        const bool empty = r0 > r1 || c0 > c1;
        C0 = c0; R0 = r0;
        nc = empty ? 0 : c1 - c0 + 1;
        nr = empty ? 0 : r1 - r0 + 1;
        const double norm = 1.0 / (2.0 * kPi * v), hv = 1.0 / (2.0 * v);
        for (int64_t j = t; j < nc; j += kT) {
            const double dx = (double)(c0 + j) - x;
            const double e = exp(-dx * dx / (2.0 * v)) * norm;
            bx[j] = e;
            bx[a.W + j] = e * dx / v;
            bx[2 * a.W + j] = e * (dx * dx / (2.0 * v * v) - hv);
        }
        for (int64_t i = t; i < nr; i += kT) {
            const double dy = (double)(r0 + i) - y;
            const double e = exp(-dy * dy / (2.0 * v));
            ay[i] = e;
            ay[a.H + i] = e * dy / v;
            ay[2 * a.H + i] = e * (dy * dy / (2.0 * v * v) - hv);
        }
    } else {
        __shared__ double u[2][kTaps], ud[2][kTaps], uw[2][kTaps];
        __shared__ double w[2][kTaps], wd[2][kTaps], ww[2][kTaps];
        const int64_t b0[2] = {(int64_t)floor(x) - 5, (int64_t)floor(y) - 5};
        if (t < 2 * kTaps) {
            const int ax = t / kTaps, k = t % kTaps;
            const double ctr = ax == 0 ? x : y;
            narrow_tap((double)(b0[ax] + k) - ctr, om, &u[ax][k], &ud[ax][k], &uw[ax][k]);
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
        const int64_t ext[2] = {a.W, a.H};
        int64_t first[2], cnt[2];
        for (int ax = 0; ax < 2; ++ax) {
            const int64_t lo = b0[ax] < 0 ? 0 : b0[ax];
            const int64_t hi = b0[ax] + kTaps - 1 > ext[ax] - 1 ? ext[ax] - 1 : b0[ax] + kTaps - 1;
            first[ax] = lo;
            cnt[ax] = hi >= lo ? hi - lo + 1 : 0;
        }
        const bool empty = cnt[0] == 0 || cnt[1] == 0;
        C0 = first[0]; R0 = first[1];
        nc = empty ? 0 : cnt[0];
        nr = empty ? 0 : cnt[1];
        if (t < nc) {
            const int k = (int)(C0 - b0[0]) + t;
            bx[t] = w[0][k]; bx[a.W + t] = wd[0][k]; bx[2 * a.W + t] = ww[0][k];
        } else if (t >= kTaps && t - kTaps < nr) {
            const int i = t - kTaps, k = (int)(R0 - b0[1]) + i;
            ay[i] = w[1][k]; ay[a.H + i] = wd[1][k]; ay[2 * a.H + i] = ww[1][k];
        }
    }
    if (t == 0) {
        const int64_t planes = final_img ? 1 : 3;
        if (check_cap && nr > 0 && planes * (a.H + nr - 1) * a.W > a.grid_cap) {
            a.st->stop = ASP_ERR_STATE;
            a.s->done = 1;
        }
        a.tapi[0] = (int32_t)C0; a.tapi[1] = (int32_t)nc;
        a.tapi[2] = (int32_t)R0; a.tapi[3] = (int32_t)nr;
    }
}

constexpr int kXB = 256;   // output columns per item of the row pass (one per thread)

// Row pass: item (y, column block) of the H + nr - 1 rows; a block of B's row
// and the taps in LDS, chunks of up to kXB taps.  NF = 3 factors for an
// evaluation, 1 for the update.
template <int NF>
__global__ __launch_bounds__(kT) void k_a4_xpass(A4Args a)
{
    if (NF == 1 ? !finished(a) : !live(a)) return;
    const int64_t C0 = a.tapi[0], nc = a.tapi[1], R0 = a.tapi[2], nr = a.tapi[3];
    if (nc == 0 || nr == 0) return;
    const int64_t W = a.W, Ny = a.H + nr - 1, plane = Ny * W;
    const int64_t yoff = a.ci - R0 - (nr - 1), xoff = a.cj - C0;
    const int64_t nxb = (W + kXB - 1) / kXB, items = Ny * nxb;
    __shared__ float seg[2 * kXB];
    __shared__ double tap[NF][kXB];
    const int t = threadIdx.x;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t y = it / nxb, ca = (it % nxb) * kXB, c = ca + t;
        const int64_t yb = y + yoff;                      // the same for the whole work-group
        double acc[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = 0.0;
        if (yb >= 0 && yb < a.Hp) {
            const float *Brow = a.psf + yb * a.Wp;
            for (int64_t j0 = 0; j0 < nc; j0 += kXB) {
                const int kx = (int)(nc - j0 < kXB ? nc - j0 : kXB);
                // seg[q] = B(yb, xb + q); output column ca + t with tap j0 + dj
                // reads q = t + kx - 1 - dj
                const int64_t xb = ca + xoff - j0 - (kx - 1);
                __syncthreads();
                for (int q = t; q < kXB + kx - 1; q += kT) {
                    const int64_t xc = xb + q;
                    seg[q] = xc >= 0 && xc < a.Wp ? Brow[xc] : 0.0f;
                }
                if (t < kx) {
#pragma unroll
                    for (int f = 0; f < NF; ++f) tap[f][t] = a.taps[f * W + j0 + t];
                }
                __syncthreads();
                for (int dj = 0; dj < kx; ++dj) {
                    const double b = (double)seg[t + kx - 1 - dj];
#pragma unroll
                    for (int f = 0; f < NF; ++f) acc[f] += tap[f][dj] * b;
                }
            }
        }
        if (c < W) {
#pragma unroll
            for (int f = 0; f < NF; ++f) a.grid[f * plane + y * W + c] = acc[f];
        }
    }
}

constexpr int kYR = 16;    // output rows per tile of the column pass (four per wave)
constexpr int kYC = 64;    // output columns per tile (one per lane)
constexpr int kYK = 32;    // row taps per chunk

// Column pass over tiles of 4 RW rows x kYC columns (work-group b takes tiles
// b, b + nblk, ...), RW = 4 rows per wave, or 1 where tiles of 16 rows would
// leave work-groups idle (small images).  Per chunk of row taps the
// work-group stages the rows of T it reaches in LDS, then wave w accumulates
// output rows RW w .. RW w + RW - 1 of its lane's column.  Then per pixel the
// sums of k_a4_gram, reduced in the same fixed order into partial row b; or,
// for the update, R -= gain F B(*)g.
template <bool Final>
__global__ __launch_bounds__(kT) void k_a4_ypass(A4Args a)
{
    if (Final ? !finished(a) : !live(a)) return;
    constexpr int NJ = Final ? 1 : 4, NP = Final ? 1 : 3;
    __shared__ double Ts[NP][kYR + kYK - 1][kYC];
    __shared__ double ts[NP][kYK];
    const int64_t nc = a.tapi[1], nr = a.tapi[3];
    const int64_t H = a.H, W = a.W;
    const bool empty = nc == 0 || nr == 0;
    const int64_t Ny = H + nr - 1, plane = Ny * W;
    const double *ay = a.taps + 3 * W;
    const double F = Final ? 0.0 : a.s->te[0];
    const double gF = Final ? a.gain * a.s->theta[0] : 0.0;
    const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
    const int64_t nxb = (W + kYC - 1) / kYC;
    const int RW = nxb * ((H + kYR - 1) / kYR) >= (int64_t)gridDim.x ? 4 : 1;
    const int TR = 4 * RW;                                 // rows per tile
    const int64_t tiles = nxb * ((H + TR - 1) / TR);
    double sums[kA4Sums];
#pragma unroll
    for (int k = 0; k < kA4Sums; ++k) sums[k] = 0.0;
    for (int64_t ti = blockIdx.x; ti < tiles; ti += gridDim.x) {
        const int64_t ra = (ti / nxb) * TR, ca = (ti % nxb) * kYC, c = ca + lane;
        double acc[4][NJ];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < NJ; ++q) acc[k][q] = 0.0;
        for (int64_t i0 = 0; !empty && i0 < nr; i0 += kYK) {
            const int kc = (int)(nr - i0 < kYK ? nr - i0 : kYK);
            // output row ra + lr with tap i0 + di reads T row ybase + ly,
            // ly = lr + kc - 1 - di
            const int64_t ybase = ra + nr - 1 - i0 - (kc - 1);
            const int nrows = TR + kc - 1;
            __syncthreads();
            // wave wq stages rows wq, wq + 4, ...: twelve loads in flight per plane
            constexpr int kU = (kYR + kYK - 1 + 3) / 4;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                double v[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int ly = wq + 4 * u;
                    const int64_t y = ybase + ly;
                    v[u] = ly < nrows && y < Ny && c < W ? a.grid[p * plane + y * W + c] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int ly = wq + 4 * u;
                    if (ly < nrows) Ts[p][ly][lane] = v[u];
                }
            }
            if (threadIdx.x < kc) {
#pragma unroll
                for (int p = 0; p < NP; ++p) ts[p][threadIdx.x] = ay[p * H + i0 + threadIdx.x];
            }
            __syncthreads();
            for (int ly = RW * wq; ly < RW * wq + RW - 1 + kc; ++ly) {
                const double t0 = Ts[0][ly][lane];
                const double t1 = Final ? 0.0 : Ts[1 % NP][ly][lane];
                const double t2 = Final ? 0.0 : Ts[2 % NP][ly][lane];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int di = RW * wq + k + kc - 1 - ly;
                    if (k < RW && di >= 0 && di < kc) {
                        const double w0 = ts[0][di];
                        acc[k][0] += w0 * t0;
                        if (!Final) {
                            acc[k][1 % NJ] += w0 * t1;
                            acc[k][2 % NJ] += ts[1 % NP][di] * t0;
                            acc[k][3 % NJ] += ts[2 % NP][di] * t0 + w0 * t2;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t r = ra + RW * wq + k;
            if (k >= RW || r >= H || c >= W) continue;
            if (Final) {
                a.R[r * W + c] = (float)((double)a.R[r * W + c] - gF * acc[k][0]);
                continue;
            }
            const double v0 = acc[k][0];
            const double J[4] = {v0, F * acc[k][1 % NJ], F * acc[k][2 % NJ], F * acc[k][3 % NJ]};
            const double D = (double)a.R[r * W + c];
            const double m = F * v0, res = D - m;
            int e = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = p; q < 4; ++q) sums[e++] += J[p] * J[q];
#pragma unroll
            for (int p = 0; p < 4; ++p) sums[10 + p] += J[p] * res;
            sums[14] += m * (m - 2.0 * D);
            sums[15] += res * res;
        }
    }
    if (Final) return;
    __shared__ double red[kT / 64][kA4Sums];
#pragma unroll
    for (int k = 0; k < kA4Sums; ++k) {
        double v = sums[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wq][k] = v;
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

hipError_t a4_trial(const A4Args &a, void *plan_inv4, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_taps, dim3(1), dim3(kT), 0, s, a, 0, 0);
    hipLaunchKernelGGL(k_a4_dft<3>, dim3(2048), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_mulsep<4>, dim3(2048), dim3(kT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecZ2D(*(hipfftHandle *)plan_inv4, (hipfftDoubleComplex *)a.spec, a.grid));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_gram, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_lm, dim3(1), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t a4_trial_direct(const A4Args &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_taps, dim3(1), dim3(kT), 0, s, a, 0, 1);
    hipLaunchKernelGGL(k_a4_xpass<3>, dim3(kA4RowBlocks), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_ypass<false>, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_lm, dim3(1), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t a4_commit(const A4Args &a, void *plan_inv, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_taps, dim3(1), dim3(kT), 0, s, a, 1, 0);
    hipLaunchKernelGGL(k_a4_dft<1>, dim3(2048), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_mulsep<1>, dim3(2048), dim3(kT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_status(hipfftExecZ2D(*(hipfftHandle *)plan_inv, (hipfftDoubleComplex *)a.spec, a.grid));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_a4_update, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_append, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t a4_commit_direct(const A4Args &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_a4_taps, dim3(1), dim3(kT), 0, s, a, 1, 1);
    hipLaunchKernelGGL(k_a4_xpass<1>, dim3(kA4RowBlocks), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_ypass<true>, dim3(a.nblk), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_a4_append, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace asp
