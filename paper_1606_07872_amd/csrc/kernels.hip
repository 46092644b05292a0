// gfx950 kernels of the Asp-Clean2016 minor cycle (Zhang, Bhatnagar, Rau &
// Zhang 2016): peak search (Sect. 2 step 1), the active-set LM fit of
// analytic Gaussians (Sect. 3, Eq. 4), the windowed residual update (Sect. 2
// step 3 with the Gaussian beam, Sect. 3 loop gain), the Gaussian fitted to
// the PSF main lobe and the Eq. 5/6 component output.
#include <float.h>
#include <math.h>

#include "asp_device.h"
#include "cycle.h"

namespace asp {

__global__ __launch_bounds__(256) void k_peak(const float *__restrict__ R, int64_t n,
                                              DevState *st)
{
    if (st->stop) return;
    peak_scan(R, n, blockIdx.x, gridDim.x, st->peak_keys);
}

hipError_t launch_peak(const Params &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_peak, dim3(grid), dim3(256), 0, s, p.R, p.H * p.W, p.st);
    return hipGetLastError();
}

// Decode the peak key and apply the stop test (step API only; the hot loop
// does this inside the fit kernel).
__global__ void k_peak_decode(Params p)
{
    __shared__ unsigned long long key_s;
    DevState *st = p.st;
    if (st->stop) return;
    const unsigned long long key = collect_peak_key(st, false, &key_s);
    if (threadIdx.x != 0) return;
    int64_t idx = (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    if (key == 0ull || idx >= p.H * p.W) { st->stop = ASP_ERR_STATE; return; }
    float v = p.R[idx];
    st->idx = idx;
    st->peak = v;
    if (fabs((double)v) < p.threshold) st->stop = ASP_STOP_THRESHOLD;
    else if (st->k >= p.max_iter) st->stop = ASP_STOP_MAXITER;
}

hipError_t launch_peak_decode(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_peak_decode, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_update(Params p)
{
    __shared__ float tab[kUpdTabFloats];
    update_tiles(p, blockIdx.x, gridDim.x, tab, true);
}

hipError_t launch_update(const Params &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

// ===========================================================================
// The Gaussian of the PSF main lobe (Sect. 3: the PSF approximated by one
// Gaussian with fixed alpha_b, omega_b).  One work-group: the peak pixel (the
// largest value, lowest index on ties), the 4-connected region around it with
// psf >= lobe_frac * peak grown by repeated sweeps, then alpha_b and omega_b
// minimising the squared error on that region (centre fixed at the peak) by
// Gauss-Newton with Marquardt damping, in FP64.
// ===========================================================================

__device__ double block_sum(double v, double *buf)
{
    const int t = threadIdx.x;
    __syncthreads();
    buf[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) buf[t] += buf[t + s];
        __syncthreads();
    }
    double r = buf[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_psf_fit(const float *__restrict__ psf, int64_t Hp,
                                                 int64_t Wp, double frac, DevState *st,
                                                 int32_t *lab)
{
    __shared__ double buf[256];
    __shared__ float pv_s[256];
    __shared__ int64_t pi_s[256];
    __shared__ int32_t changed;
    __shared__ double th[2], mu_s, Fcur;
    __shared__ int32_t flag, stop;
    const int t = threadIdx.x;
    const int64_t n = Hp * Wp;
    float bv = -FLT_MAX;
    int64_t bi = 0;
    for (int64_t i = t; i < n; i += 256)
        if (psf[i] > bv) { bv = psf[i]; bi = i; }
    pv_s[t] = bv;
    pi_s[t] = bi;
    __syncthreads();
    if (t == 0) {
        float b = pv_s[0];
        int64_t ib = pi_s[0];
        for (int i = 1; i < 256; ++i)
            if (pv_s[i] > b || (pv_s[i] == b && pi_s[i] < ib)) { b = pv_s[i]; ib = pi_s[i]; }
        pv_s[0] = b;
        pi_s[0] = ib;
        st->psf_status = (b > 0.0f) ? 0 : ASP_ERR_PSF;
    }
    __syncthreads();
    const double pv = pv_s[0];
    const int64_t pk = pi_s[0];
    if (!(pv > 0.0)) return;
    const double lim = frac * pv;
    for (int64_t i = t; i < n; i += 256) lab[i] = ((double)psf[i] >= lim) ? 1 : 0;
    __syncthreads();
    if (t == 0) lab[pk] = 2;
    __syncthreads();
    do {
        __syncthreads();
        if (t == 0) changed = 0;
        __syncthreads();
        for (int64_t i = t; i < n; i += 256) {
            if (lab[i] != 1) continue;
            int64_t r = i / Wp, c = i % Wp;
            if ((r > 0 && lab[i - Wp] == 2) || (r < Hp - 1 && lab[i + Wp] == 2) ||
                (c > 0 && lab[i - 1] == 2) || (c < Wp - 1 && lab[i + 1] == 2)) {
                lab[i] = 2;
                changed = 1;
            }
        }
        __threadfence_block();
        __syncthreads();
    } while (changed);
    const int64_t pr = pk / Wp, pc = pk % Wp;
    double cnt = 0.0;
    for (int64_t i = t; i < n; i += 256) cnt += (lab[i] == 2) ? 1.0 : 0.0;
    const double nl = block_sum(cnt, buf);
    if (t == 0) {
        th[0] = pv;
        th[1] = (nl > 1.0) ? sqrt(nl / (2.0 * M_PI * log(1.0 / frac))) : 0.5;
        mu_s = 1e-3;
        stop = 0;
    }
    __syncthreads();
    for (int it = 0; it < 500 && !stop; ++it) {
        const double a = th[0], w = th[1], w2 = w * w;
        double F = 0, h00 = 0, h01 = 0, h11 = 0, g0 = 0, g1 = 0;
        for (int64_t i = t; i < n; i += 256) {
            if (lab[i] != 2) continue;
            double dr = (double)(i / Wp - pr), dc = (double)(i % Wp - pc);
            double q = dr * dr + dc * dc;
            double e = exp(-q / (2.0 * w2));
            double G = a * e;
            double j0 = e, j1 = G * q / (w2 * w);
            double r = (double)psf[i] - G;
            F += r * r; h00 += j0 * j0; h01 += j0 * j1; h11 += j1 * j1;
            g0 += j0 * r; g1 += j1 * r;
        }
        F = block_sum(F, buf); h00 = block_sum(h00, buf); h01 = block_sum(h01, buf);
        h11 = block_sum(h11, buf); g0 = block_sum(g0, buf); g1 = block_sum(g1, buf);
        if (t == 0) {
            if (it == 0) Fcur = F;
            flag = 0;   // 0: still damping, 1: accepted, 2: give up
        }
        __syncthreads();
        while (true) {
            __shared__ double tr[2];
            if (t == 0) {
                if (mu_s > 1e8) { flag = 2; }
                else {
                    double A00 = h00 * (1.0 + mu_s), A11 = h11 * (1.0 + mu_s), A01 = h01;
                    double det = A00 * A11 - A01 * A01;
                    if (!(A00 > 0.0) || !(det > 0.0)) { mu_s *= 10.0; flag = 3; }
                    else {
                        double d0 = (A11 * g0 - A01 * g1) / det;
                        double d1 = (A00 * g1 - A01 * g0) / det;
                        tr[0] = a + d0;
                        tr[1] = w + d1;
                        if (!(tr[1] > 1e-3)) tr[1] = 1e-3;
                        flag = 0;
                    }
                }
            }
            __syncthreads();
            if (flag == 2) break;
            if (flag == 3) continue;
            const double ta = tr[0], tw = tr[1];
            double Ft = 0.0;
            for (int64_t i = t; i < n; i += 256) {
                if (lab[i] != 2) continue;
                double dr = (double)(i / Wp - pr), dc = (double)(i % Wp - pc);
                double r = (double)psf[i] - ta * exp(-(dr * dr + dc * dc) / (2.0 * tw * tw));
                Ft += r * r;
            }
            Ft = block_sum(Ft, buf);
            if (t == 0) {
                if (isfinite(Ft) && Ft < Fcur) {
                    double step = fabs(ta - a) / fabs(ta) + fabs(tw - w) / tw;
                    th[0] = ta; th[1] = tw; Fcur = Ft;
                    mu_s = mu_s / 10.0 < 1e-12 ? 1e-12 : mu_s / 10.0;
                    flag = 1;
                    if (step < 1e-14) stop = 1;
                } else {
                    mu_s *= 10.0;
                    flag = 0;
                }
            }
            __syncthreads();
            if (flag == 1) break;
        }
        if (t == 0 && flag == 2) stop = 1;
        __syncthreads();
    }
    if (t == 0) {
        st->alpha_b = th[0];
        st->omega_b = th[1];
        st->lobe_px = (int64_t)nl;
    }
}

hipError_t launch_psf_fit(const float *psf, int64_t Hp, int64_t Wp, double lobe_frac,
                          DevState *st, int32_t *work, hipStream_t s)
{
    hipLaunchKernelGGL(k_psf_fit, dim3(1), dim3(256), 0, s, psf, Hp, Wp, lobe_frac, st, work);
    return hipGetLastError();
}

__global__ void k_check_finite(const float *__restrict__ img, int64_t n, int32_t *flag)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(img[i])) { atomicOr(flag, 1); return; }
}

hipError_t launch_check_finite(const float *img, int64_t n, int32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, s, img, n, flag);
    return hipGetLastError();
}

// Sum of squares of an image in FP64, in a fixed order: per-work-group
// partials (grid-strided, float4), then one work-group sums them in order.
__global__ __launch_bounds__(256) void k_sumsq_part(const float *__restrict__ img, int64_t n,
                                                    double *part)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int64_t n4 = n >> 2;
    const float4 *v4 = reinterpret_cast<const float4 *>(img);
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + t; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = v4[i];
        s += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    }
    if (blockIdx.x == 0 && t < (int)(n - 4 * n4)) s += (double)img[4 * n4 + t] * img[4 * n4 + t];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sumsq_final(const double *part, int n, double *out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
}

hipError_t launch_sumsq(const float *img, int64_t n, double *part, int nblk, double *out,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_sumsq_part, dim3(nblk), dim3(256), 0, s, img, n, part);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, s, part, nblk, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sq_rebase(DevState *st, const double *total)
{
    for (int i = threadIdx.x; i < st->sq_nslots; i += blockDim.x) st->sq_slots[i] = 0.0;
    if (threadIdx.x == 0) st->sq_base = *total;
}

// base + slot sums: thread t adds slots t, t + 256, ...; then the 256 sums in order
__global__ __launch_bounds__(256) void k_sq_read(DevState *st, double *out)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < st->sq_nslots; i += blockDim.x) v += st->sq_slots[i];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = st->sq_base;
        for (int i = 0; i < 256; ++i) sum += red[i];
        *out = sum;
    }
}

// the pixel counts: integer sums, exact in any order
__global__ __launch_bounds__(256) void k_px_read(DevState *st)
{
    __shared__ unsigned long long red[256];
    unsigned long long v = 0;
    for (int i = threadIdx.x; i < st->sq_nslots; i += blockDim.x) v += st->px_slots[i];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int i = 0; i < 256; ++i) sum += red[i];
        st->px_total = sum;
    }
}

hipError_t launch_px_read(DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_px_read, dim3(1), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_sq_rebase(DevState *st, const double *total, hipStream_t s)
{
    hipLaunchKernelGGL(k_sq_rebase, dim3(1), dim3(256), 0, s, st, total);
    return hipGetLastError();
}

hipError_t launch_sq_read(DevState *st, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sq_read, dim3(1), dim3(256), 0, s, st, out);
    return hipGetLastError();
}

// Eqs. 5-6: sky-plane parameters of every component.
__global__ void k_components(Params p, asp_component *out)
{
    const DevState *st = p.st;
    const int64_t L = st->L;
    const double ab = st->alpha_b, wb = st->omega_b;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < L;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double a = p.ca[j], s = p.cs[j];
        double w2 = s * s - wb * wb;
        if (w2 < 0.0) w2 = 0.0;
        const double w = sqrt(w2);
        asp_component c;
        c.flux = a * s * s / (ab * wb * wb);                      // 2 pi alpha_i omega_i^2
        c.width = w;                                              // Eq. 5
        c.is_point = (w > 1e-6 * wb) ? 0 : 1;
        c.amp = c.is_point ? 0.0 : a * s * s / (2.0 * M_PI * ab * wb * wb * w2);   // Eq. 6
        c.x = p.cx[j];
        c.y = p.cy[j];
        c.amp_c = a;
        c.width_c = s;
        c.pad = 0;
        c.iter_added = p.c_added[j];
        c.iter_updated = p.c_updated[j];
        out[j] = c;
    }
}

hipError_t launch_components(const Params &p, asp_component *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_components, dim3(64), dim3(256), 0, s, p, out);
    return hipGetLastError();
}

}  // namespace asp
