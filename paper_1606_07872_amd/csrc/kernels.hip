// gfx950 kernels of the Asp-Clean2016 minor cycle (Zhang, Bhatnagar, Rau &
// Zhang 2016): peak search (Sect. 2 step 1), the active-set LM fit of
// analytic Gaussians (Sect. 3, Eq. 4), the windowed residual update (Sect. 2
// step 3 with the Gaussian beam, Sect. 3 loop gain), the Gaussian fitted to
// the PSF main lobe and the Eq. 5/6 component output.
#include <float.h>
#include <math.h>

#include "asp_device.h"

namespace asp {

// ===========================================================================
// Peak search: the largest |R|, the lowest row-major index winning ties.
// Each thread walks its elements in increasing index order keeping the first
// strict maximum; the block combines packed keys (|v| bits << 32 | ~idx), whose
// integer maximum is exactly that rule, and one 64-bit atomicMax per block
// makes the result independent of block order.
// ===========================================================================

__device__ inline void peak_take(float v, uint32_t i, float &bv, uint32_t &bi)
{
    float a = fabsf(v);
    if (a > bv) { bv = a; bi = i; }
}

__device__ inline void peak_take4(const float4 &v, uint32_t i4, float &bv, uint32_t &bi)
{
    peak_take(v.x, 4 * i4 + 0, bv, bi);
    peak_take(v.y, 4 * i4 + 1, bv, bi);
    peak_take(v.z, 4 * i4 + 2, bv, bi);
    peak_take(v.w, 4 * i4 + 3, bv, bi);
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_peak(const float *__restrict__ R, int64_t n,
                                              DevState *st)
{
    if (st->stop) return;
    const uint32_t n4 = (uint32_t)(n >> 2);
    const float4 *R4 = reinterpret_cast<const float4 *>(R);
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    float bv = -1.0f;
    uint32_t bi = 0;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        float4 v0 = R4[i], v1 = R4[i + stride], v2 = R4[i + 2 * stride], v3 = R4[i + 3 * stride];
        peak_take4(v0, i, bv, bi);
        peak_take4(v1, i + stride, bv, bi);
        peak_take4(v2, i + 2 * stride, bv, bi);
        peak_take4(v3, i + 3 * stride, bv, bi);
    }
    for (; i < n4; i += stride) peak_take4(R4[i], i, bv, bi);
    uint32_t tail = (uint32_t)(n - 4 * (int64_t)n4);
    if (blockIdx.x == 0 && threadIdx.x < tail) {
        uint32_t j = 4 * n4 + threadIdx.x;
        peak_take(R[j], j, bv, bi);
    }
    unsigned long long key = 0;
    if (bv >= 0.0f)
        key = ((unsigned long long)__float_as_uint(bv) << 32) | (unsigned long long)(0xFFFFFFFFu - bi);
    key = wave_max_u64(key);
    __shared__ unsigned long long wk[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wk[wave] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = wk[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) k = wk[w] > k ? wk[w] : k;
        atomicMax(&st->peak_key, k);
    }
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
    DevState *st = p.st;
    if (st->stop) return;
    unsigned long long key = st->peak_key;
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
    hipLaunchKernelGGL(k_peak_decode, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

// ===========================================================================
// Residual update: R += sum over the plan's rects of sign * G on the rect,
// each pixel read and written once (Sect. 2 step 3 with the Gaussian beam).
// Blocks stride over 64 x 4 tiles of the plan's bounding box and skip tiles
// that meet no rect.
// ===========================================================================

__global__ __launch_bounds__(256) void k_update(Params p)
{
    DevState *st = p.st;
    if (!st->fit_ready) return;
    __shared__ int32_t rb[kMaxRects][4];
    __shared__ int32_t rcx[kMaxRects], rcy[kMaxRects];
    __shared__ float rfx[kMaxRects], rfy[kMaxRects], ramp[kMaxRects], rinv[kMaxRects];
    __shared__ int32_t nr_s, bb_s[4];
    __shared__ unsigned long long cnt_s[4];
    const int t = threadIdx.x;
    if (t == 0) {
        nr_s = st->n_rects;
        for (int i = 0; i < 4; ++i) bb_s[i] = st->bb[i];
    }
    if (t < st->n_rects) {
        const Rect &R = st->rects[t];
        rb[t][0] = R.r0; rb[t][1] = R.r1; rb[t][2] = R.c0; rb[t][3] = R.c1;
        double cx = floor(R.x + 0.5), cy = floor(R.y + 0.5);
        rcx[t] = (int32_t)cx;
        rcy[t] = (int32_t)cy;
        rfx[t] = (float)(R.x - cx);
        rfy[t] = (float)(R.y - cy);
        ramp[t] = (float)((double)R.sign * R.a);
        rinv[t] = (float)(1.0 / (2.0 * R.s * R.s));
    }
    __syncthreads();
    const int nr = nr_s;
    const int32_t br0 = bb_s[0], br1 = bb_s[1], bc0 = bb_s[2], bc1 = bb_s[3];
    const int ntx = (bc1 - bc0 + 64) / 64, nty = (br1 - br0 + 4) / 4;
    const int64_t ntiles = (int64_t)ntx * nty;
    unsigned long long cnt = 0;
    const int lr = t >> 6, lc = t & 63;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int32_t tr0 = br0 + (int32_t)(tile / ntx) * 4;
        const int32_t tc0 = bc0 + (int32_t)(tile % ntx) * 64;
        bool any = false;
        for (int i = 0; i < nr; ++i)
            any |= (rb[i][0] <= tr0 + 3 && tr0 <= rb[i][1] && rb[i][2] <= tc0 + 63 && tc0 <= rb[i][3]);
        if (!any) continue;
        const int32_t r = tr0 + lr, c = tc0 + lc;
        if (r > br1 || c > bc1) continue;
        float acc = 0.0f;
        bool hit = false;
        for (int i = 0; i < nr; ++i) {
            if (r < rb[i][0] || r > rb[i][1] || c < rb[i][2] || c > rb[i][3]) continue;
            float dx = (float)(c - rcx[i]) - rfx[i];
            float dy = (float)(r - rcy[i]) - rfy[i];
            acc += ramp[i] * __expf(-(dx * dx + dy * dy) * rinv[i]);
            hit = true;
        }
        if (hit) {
            float *px = p.R + (int64_t)r * p.W + c;
            *px = *px + acc;
            ++cnt;
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((t & 63) == 0) cnt_s[t >> 6] = cnt;
    __syncthreads();
    if (t == 0) {
        unsigned long long c = cnt_s[0] + cnt_s[1] + cnt_s[2] + cnt_s[3];
        if (c) {
            atomicAdd(&st->update_px, c);
            atomicAdd(&st->sum_update_px, c);
        }
    }
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
