// Exact-PSF residual refresh (Sect. 2 step 3): R = I_dirty - B (*) I_model with
// the true PSF B, replacing the residual that the minor cycle keeps by
// subtracting each component's Gaussian main-lobe approximation (Sect. 3).
//
// The model image is rendered from the component list (Eqs. 5-6: flux,
// width, centre) into a zero-padded FP64 grid, tile by tile, each tile
// gathering the components that meet it: components at least 1 px wide
// as sampled Gaussians on their windows; narrower ones (points included) by
// band-limited interpolation -- per axis the 3-point Gauss-Hermite rule of
// the Gaussian (offsets 0, +-sqrt(3) omega; weights 2/3, 1/6, 1/6), each node
// spread with the Lanczos-3 kernel, the weights normalised to sum 1.  The
// linear convolution with the PSF (centred on its peak pixel) is a product of
// spectra: hipFFT for the two real transforms (FP64), the PSF's spectrum
// computed once.  Rendering, spectral product and the subtraction are the
// kernels below.
#include <hipfft/hipfft.h>

#include "asp_device.h"

namespace asp {
namespace {

constexpr int kT = 256;
constexpr int kTaps = 12;           // per-axis taps of the interpolated profile

__device__ inline bool refresh_on(const RefreshArgs &a)
{
    return a.force || a.st->stop == 0;
}

__global__ __launch_bounds__(kT) void k_rf_zero(RefreshArgs a)
{
    const int64_t n = a.Py * a.Px;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        a.grid[i] = 0.0;
}

__global__ __launch_bounds__(kT) void k_rf_psf(RefreshArgs a)
{
    const int64_t n = a.Hp * a.Wp;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const int64_t r = i / a.Wp, c = i % a.Wp;
        a.grid[r * a.Px + c] = (double)a.psf[i];
    }
}

__device__ inline double lanczos3(double t)
{
    if (t == 0.0) return 1.0;
    if (!(fabs(t) < 3.0)) return 0.0;
    const double pt = 3.14159265358979323846 * t;
    return (sinpi(t) / pt) * (sinpi(t / 3.0) / (pt / 3.0));
}

// The rendering of one component, as the tile needs it.
struct Comp {
    double amp, x, y;              // alpha (wide) or flux (narrow); the centre
    double inv, d1;                // 1 / (2 omega^2) (wide); sqrt(3) omega (narrow)
    int64_t r0, r1, c0, c1;        // its footprint (wide: the window, not clipped)
    bool wide;
};

// Eqs. (5)-(6) and the footprint of component j.
__device__ inline Comp component(const RefreshArgs &a, int64_t j, double alpha_b, double omega_b)
{
    Comp q;
    const double amp = a.ca[j], x = a.cx[j], y = a.cy[j], s = a.cs[j];
    const double flux = __ddiv_rn(__dmul_rn(__dmul_rn(amp, s), s),
                                  __dmul_rn(__dmul_rn(alpha_b, omega_b), omega_b));
    const double w2 = __dsub_rn(__dmul_rn(s, s), __dmul_rn(omega_b, omega_b));
    const double omega = w2 > 0.0 ? sqrt(w2) : 0.0;
    const bool point = !(omega > 1e-6 * omega_b);
    q.x = x;
    q.y = y;
    q.wide = !point && omega >= 1.0;
    if (q.wide) {
        q.amp = flux / (2.0 * 3.14159265358979323846 * omega * omega);
        q.inv = 1.0 / (2.0 * omega * omega);
        q.d1 = 0.0;
        const int64_t h = halfwidth(omega, a.window_sigmas);
        const int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
        q.r0 = cy - h; q.r1 = cy + h; q.c0 = cx - h; q.c1 = cx + h;
    } else {
        q.amp = flux;
        q.inv = 0.0;
        q.d1 = 1.7320508075688772 * (point ? 0.0 : omega);      // sqrt(3) omega
        q.c0 = (int64_t)floor(x) - 5; q.c1 = q.c0 + kTaps - 1;
        q.r0 = (int64_t)floor(y) - 5; q.r1 = q.r0 + kTaps - 1;
    }
    return q;
}

__device__ inline double gh_lanczos(double u, double d1)
{
    return (2.0 / 3.0) * lanczos3(u) + (1.0 / 6.0) * lanczos3(u - d1) + (1.0 / 6.0) * lanczos3(u + d1);
}

// Work-group per 64 x 64 tile of the image: every component whose footprint
// meets the tile is added into registers, in the order of the component
// list (no atomics; the sum has a fixed order), and the tile is written once.
// Lane = column, wave w = rows w, w + 4, ...
__global__ __launch_bounds__(kT) void k_rf_render(RefreshArgs a)
{
    if (!refresh_on(a)) return;
    constexpr int TS = 64, RPT = TS / (kT / 64);
    const DevState *st = a.st;
    const int64_t L = st->L;
    const double alpha_b = st->alpha_b, omega_b = st->omega_b;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tx = (a.W + TS - 1) / TS;
    const int64_t tr0 = (int64_t)(blockIdx.x / tx) * TS, tc0 = (int64_t)(blockIdx.x % tx) * TS;
    const int64_t tr1 = (tr0 + TS < a.H ? tr0 + TS : a.H) - 1, tc1 = (tc0 + TS < a.W ? tc0 + TS : a.W) - 1;
    __shared__ int64_t hits[kT];
    __shared__ int wave_n[kT / 64];
    __shared__ double fx[TS], fy[TS];
    __shared__ double nsum[2];
    double acc[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) acc[k] = 0.0;
    const int64_t c = tc0 + lane;
    for (int64_t base = 0; base < L; base += kT) {
        // the components base .. base + 255 that meet the tile, in order
        const int64_t j = base + t;
        bool hit = false;
        if (j < L) {
            const Comp q = component(a, j, alpha_b, omega_b);
            hit = q.r0 <= tr1 && q.r1 >= tr0 && q.c0 <= tc1 && q.c1 >= tc0;
        }
        const unsigned long long m = __ballot(hit);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        __syncthreads();                   // hits of the previous chunk are consumed
        if (lane == 0) wave_n[w] = __popcll(m);
        __syncthreads();
        int off = 0, n = 0;
        for (int v = 0; v < kT / 64; ++v) {
            off += v < w ? wave_n[v] : 0;
            n += wave_n[v];
        }
        if (hit) hits[off + before] = j;
        __syncthreads();
        for (int e = 0; e < n; ++e) {
            const Comp q = component(a, hits[e], alpha_b, omega_b);
            if (q.wide) {
                // row and column factors of the window, zero outside it
                if (t < TS) {
                    const int64_t cc = tc0 + t;
                    const double d = (double)cc - q.x;
                    fx[t] = (cc >= q.c0 && cc <= q.c1) ? exp(-(d * d) * q.inv) : 0.0;
                } else if (t < 2 * TS) {
                    const int64_t rr = tr0 + (t - TS);
                    const double d = (double)rr - q.y;
                    fy[t - TS] = (rr >= q.r0 && rr <= q.r1) ? exp(-(d * d) * q.inv) : 0.0;
                }
                __syncthreads();
                const double vx = q.amp * fx[lane];
#pragma unroll
                for (int k = 0; k < RPT; ++k) acc[k] += vx * fy[w + (kT / 64) * k];
            } else {
                // per-axis weights of the interpolated profile, normalised
                if (t < TS) {
                    const int64_t cc = tc0 + t;
                    fx[t] = (cc >= q.c0 && cc <= q.c1) ? gh_lanczos((double)cc - q.x, q.d1) : 0.0;
                } else if (t < 2 * TS) {
                    const int64_t rr = tr0 + (t - TS);
                    fy[t - TS] = (rr >= q.r0 && rr <= q.r1) ? gh_lanczos((double)rr - q.y, q.d1) : 0.0;
                } else if (t < 2 * TS + 2) {
                    // the sums over the whole 12 taps, inside the image or not
                    const bool ax = t == 2 * TS;
                    const int64_t b0 = ax ? q.c0 : q.r0;
                    const double ctr = ax ? q.x : q.y;
                    double sum = 0.0;
                    for (int k = 0; k < kTaps; ++k) sum += gh_lanczos((double)(b0 + k) - ctr, q.d1);
                    nsum[ax ? 0 : 1] = sum;
                }
                __syncthreads();
                const double vx = q.amp * (fx[lane] / nsum[0]);
#pragma unroll
                for (int k = 0; k < RPT; ++k) acc[k] += vx * (fy[w + (kT / 64) * k] / nsum[1]);
            }
            __syncthreads();               // fx, fy are rewritten by the next entry
        }
    }
    if (c <= tc1) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int64_t r = tr0 + w + (kT / 64) * k;
            if (r <= tr1) a.grid[r * a.Px + c] = acc[k];
        }
    }
}

// The model's spectrum times the PSF's, with the 1 / (Py Px) of the inverse.
__global__ __launch_bounds__(kT) void k_rf_mul(RefreshArgs a)
{
    const int64_t n = a.Py * (a.Px / 2 + 1);
    const double scale = 1.0 / ((double)a.Py * (double)a.Px);
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const double2 m = a.spec[i], b = a.pspec[i];
        a.spec[i] = make_double2((m.x * b.x - m.y * b.y) * scale, (m.x * b.y + m.y * b.x) * scale);
    }
}

// R(r, c) = D(r, c) - (B (*) M)(r + ci, c + cj) of the full linear convolution.
__global__ __launch_bounds__(kT) void k_rf_finish(RefreshArgs a)
{
    if (!refresh_on(a)) return;
    const int64_t n = a.H * a.W;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const int64_t r = i / a.W, c = i % a.W;
        a.R[i] = (float)((double)a.dirty[i] - a.grid[(r + a.ci) * a.Px + (c + a.cj)]);
    }
}

// The image part of the rendered model, rounded to FP32.
__global__ __launch_bounds__(kT) void k_rf_model_out(RefreshArgs a, float *out)
{
    for (int64_t r = blockIdx.x; r < a.H; r += gridDim.x)
        for (int64_t c = threadIdx.x; c < a.W; c += kT) out[r * a.W + c] = (float)a.grid[r * a.Px + c];
}

hipError_t fft_error(hipfftResult r)
{
    return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown;
}

}  // namespace

hipError_t refresh_psf_spectrum(const RefreshArgs &a, void *plan_fwd, hipStream_t s)
{
    hipLaunchKernelGGL(k_rf_zero, dim3(2048), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_rf_psf, dim3(256), dim3(kT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return fft_error(hipfftExecD2Z(*(hipfftHandle *)plan_fwd, a.grid,
                                   (hipfftDoubleComplex *)a.pspec));
}

hipError_t refresh_residual(const RefreshArgs &a, void *plan_fwd, void *plan_inv, hipStream_t s)
{
    hipLaunchKernelGGL(k_rf_zero, dim3(2048), dim3(kT), 0, s, a);
    const int64_t tiles = ((a.H + 63) / 64) * ((a.W + 63) / 64);
    hipLaunchKernelGGL(k_rf_render, dim3((unsigned)tiles), dim3(kT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_error(hipfftExecD2Z(*(hipfftHandle *)plan_fwd, a.grid, (hipfftDoubleComplex *)a.spec));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rf_mul, dim3(2048), dim3(kT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = fft_error(hipfftExecZ2D(*(hipfftHandle *)plan_inv, (hipfftDoubleComplex *)a.spec, a.grid));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rf_finish, dim3(2048), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t render_model(const RefreshArgs &a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_rf_zero, dim3(2048), dim3(kT), 0, s, a);
    const int64_t tiles = ((a.H + 63) / 64) * ((a.W + 63) / 64);
    hipLaunchKernelGGL(k_rf_render, dim3((unsigned)tiles), dim3(kT), 0, s, a);
    const int64_t rows = a.H < 4096 ? a.H : 4096;
    hipLaunchKernelGGL(k_rf_model_out, dim3((unsigned)rows), dim3(kT), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace asp
