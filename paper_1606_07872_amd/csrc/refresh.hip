// Exact-PSF residual refresh (Sect. 2 step 3): R = I_dirty - B (*) I_model with
// the true PSF B, replacing the residual that the minor cycle keeps by
// subtracting each component's Gaussian main-lobe approximation (Sect. 3).
//
// The model image is rendered from the component list (Eqs. 5-6: flux,
// width, centre) into a zero-padded FP64 grid: components at least 1 px wide
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
constexpr int kRenderGrid = 1024;
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

// Work-group per component (grid-stride over the list); FP64 atomics into the
// padded grid, whose first H rows and W columns hold the image.
__global__ __launch_bounds__(kT) void k_rf_render(RefreshArgs a)
{
    if (!refresh_on(a)) return;
    const DevState *st = a.st;
    const int64_t L = st->L;
    const double alpha_b = st->alpha_b, omega_b = st->omega_b;
    const int t = threadIdx.x;
    __shared__ double wx[kTaps], wy[kTaps];
    __shared__ double sums[2];
    for (int64_t j = blockIdx.x; j < L; j += gridDim.x) {
        const double amp = a.ca[j], x = a.cx[j], y = a.cy[j], s = a.cs[j];
        // Eqs. (5)-(6)
        const double flux = __ddiv_rn(__dmul_rn(__dmul_rn(amp, s), s),
                                      __dmul_rn(__dmul_rn(alpha_b, omega_b), omega_b));
        const double w2 = __dsub_rn(__dmul_rn(s, s), __dmul_rn(omega_b, omega_b));
        const double omega = w2 > 0.0 ? sqrt(w2) : 0.0;
        const bool point = !(omega > 1e-6 * omega_b);
        __syncthreads();                   // LDS of the previous component is read
        if (!point && omega >= 1.0) {
            const double alpha = flux / (2.0 * 3.14159265358979323846 * omega * omega);
            const double inv = 1.0 / (2.0 * omega * omega);
            const int64_t h = halfwidth(omega, a.window_sigmas);
            const int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
            const int64_t r0 = cy - h > 0 ? cy - h : 0, r1 = cy + h < a.H - 1 ? cy + h : a.H - 1;
            const int64_t c0 = cx - h > 0 ? cx - h : 0, c1 = cx + h < a.W - 1 ? cx + h : a.W - 1;
            if (r0 > r1 || c0 > c1) continue;
            const int64_t nc = c1 - c0 + 1, np = (r1 - r0 + 1) * nc;
            for (int64_t q = t; q < np; q += kT) {
                const int64_t r = r0 + q / nc, c = c0 + q % nc;
                const double dx = (double)c - x, dy = (double)r - y;
                atomicAdd(&a.grid[r * a.Px + c], alpha * exp(-(dx * dx + dy * dy) * inv));
            }
        } else {
            const double om = point ? 0.0 : omega;
            const double d1 = 1.7320508075688772 * om;     // sqrt(3) omega
            const int64_t bx = (int64_t)floor(x) - 5, by = (int64_t)floor(y) - 5;
            if (t < 2 * kTaps) {
                const bool ax = t < kTaps;
                const int k = ax ? t : t - kTaps;
                const double u = ax ? (double)(bx + k) - x : (double)(by + k) - y;
                const double v = (2.0 / 3.0) * lanczos3(u) + (1.0 / 6.0) * lanczos3(u - d1) +
                                 (1.0 / 6.0) * lanczos3(u + d1);
                (ax ? wx : wy)[k] = v;
            }
            __syncthreads();
            if (t < 2) {
                const double *w = t == 0 ? wx : wy;
                double acc = 0.0;
                for (int k = 0; k < kTaps; ++k) acc += w[k];
                sums[t] = acc;
            }
            __syncthreads();
            if (t < kTaps * kTaps) {
                const int i = t / kTaps, k = t % kTaps;
                const int64_t r = by + i, c = bx + k;
                if (r >= 0 && r < a.H && c >= 0 && c < a.W)
                    atomicAdd(&a.grid[r * a.Px + c], flux * (wy[i] / sums[1]) * (wx[k] / sums[0]));
            }
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
    hipLaunchKernelGGL(k_rf_render, dim3(kRenderGrid), dim3(kT), 0, s, a);
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

}  // namespace asp
