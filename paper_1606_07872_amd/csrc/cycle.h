// Device functions of the minor cycle shared by the single-field kernels
// (one launch per step, the whole grid on one field) and the batched kernel
// (a team of work-groups per field): the peak search and the windowed
// residual update, each over the share `rank` of `size` work-groups.
#pragma once

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

// The work-group's key goes to slots[rank % kPeakSlots] (a 64-bit atomicMax);
// the peak is the maximum over the kPeakSlots slots.
__device__ inline void peak_scan(const float *__restrict__ R, int64_t n, uint32_t rank,
                                 uint32_t size, unsigned long long *slots)
{
    const uint32_t n4 = (uint32_t)(n >> 2);
    const float4 *R4 = reinterpret_cast<const float4 *>(R);
    const uint32_t stride = size * blockDim.x;
    uint32_t i = rank * blockDim.x + threadIdx.x;
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
    if (rank == 0 && threadIdx.x < tail) {
        uint32_t j = 4 * n4 + threadIdx.x;
        peak_take(R[j], j, bv, bi);
    }
    unsigned long long key = 0;
    if (bv >= 0.0f)
        key = ((unsigned long long)__float_as_uint(bv) << 32) | (unsigned long long)(0xFFFFFFFFu - bi);
    key = wave_max_u64(key);
    __shared__ unsigned long long wk[4];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wk[wave] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long k = wk[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) k = wk[w] > k ? wk[w] : k;
        atomicMax(&slots[rank % kPeakSlots], k);
    }
}

// ===========================================================================
// Residual update: R += sum over the plan's rects of sign * G on the rect,
// each pixel read and written once (Sect. 2 step 3 with the Gaussian beam).
// Blocks stride over 64 x 16 tiles of the plan's bounding box and skip tiles
// that meet no rect.
// ===========================================================================

__device__ inline void update_tiles(const Params &p, int rank, int size)
{
    DevState *st = p.st;
    __shared__ int32_t rb[kMaxRects][4];
    __shared__ int32_t rcx[kMaxRects], rcy[kMaxRects];
    __shared__ float rfx[kMaxRects], rfy[kMaxRects], ramp[kMaxRects], rinv[kMaxRects];
    __shared__ int32_t nr_s, bb_s[4];
    __shared__ unsigned long long cnt_s[4];
    __shared__ double dsq_s[4];
    const int t = threadIdx.x;
    __syncthreads();
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
    // tiles of 64 columns x kUpdRows rows; a thread takes column lc of rows
    // lr, lr + 4, ...: its kUpdRows / 4 pixels are loaded together, so that a
    // wave keeps several loads in flight
    constexpr int kUpdRows = 16, kPer = kUpdRows / 4;
    const int ntx = (bc1 - bc0 + 64) / 64, nty = (br1 - br0 + kUpdRows) / kUpdRows;
    // a bounding box lies inside the image (fewer than 2^32 pixels), so tile
    // indices fit in 32 bits
    const int32_t ntiles = ntx * nty;
    static_assert(kMaxRects <= 32, "one bit per rect");
    uint32_t cnt32 = 0;
    double dsq = 0.0;                   // change of the sum of R^2 over this thread's pixels
    const int lr = t >> 6, lc = t & 63;
    const int64_t rstride = 4 * (int64_t)p.W;   // rows lr, lr + 4, ... of a tile
    for (int32_t tile = rank; tile < ntiles; tile += size) {
        const int32_t ty = tile / ntx;
        const int32_t tr0 = br0 + ty * kUpdRows;
        const int32_t tc0 = bc0 + (tile - ty * ntx) * 64;
        bool any = false;
        for (int i = 0; i < nr; ++i)
            any |= (rb[i][0] <= tr0 + kUpdRows - 1 && tr0 <= rb[i][1] && rb[i][2] <= tc0 + 63 &&
                    tc0 <= rb[i][3]);
        if (!any) continue;
        const int32_t c = tc0 + lc;
        if (c > bc1) continue;
        // the rects whose columns hold this thread's column (fixed in a tile)
        uint32_t colmask = 0u;
        for (int i = 0; i < nr; ++i)
            colmask |= (c >= rb[i][2] && c <= rb[i][3]) ? (1u << i) : 0u;
        const int64_t q = (int64_t)(tr0 + lr) * p.W + c;   // pixel k at q + k * rstride
        float acc[kPer], val[kPer];
        bool hit[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int32_t r = tr0 + lr + 4 * k;
            acc[k] = 0.0f;
            hit[k] = false;
            if (r > br1) continue;
            for (int i = 0; i < nr; ++i)
                hit[k] |= ((colmask >> i) & 1u) && r >= rb[i][0] && r <= rb[i][1];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) val[k] = hit[k] ? p.R[q + k * rstride] : 0.0f;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (!hit[k]) continue;
            const int32_t r = tr0 + lr + 4 * k;
            for (int i = 0; i < nr; ++i) {
                if (!((colmask >> i) & 1u) || r < rb[i][0] || r > rb[i][1]) continue;
                float dx = (float)(c - rcx[i]) - rfx[i];
                float dy = (float)(r - rcy[i]) - rfy[i];
                acc[k] += ramp[i] * __expf(-(dx * dx + dy * dy) * rinv[i]);
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (!hit[k]) continue;
            const float nv = val[k] + acc[k];
            p.R[q + k * rstride] = nv;
            dsq += (double)nv * nv - (double)val[k] * val[k];
            ++cnt32;
        }
    }
    unsigned long long cnt = cnt32;
    if (p.sm.n > 0 && rank == 0) {
        // tiles of the smoothed images that these windows make stale: per
        // scale j, rows within h_j of a window for the column pass, rows and
        // columns within h_j for the row pass
        const int tx = p.sm.tiles_x, ty = p.sm.tiles_y;
        const int64_t ntl = (int64_t)tx * ty;
        for (int pair = 0; pair < nr * p.sm.n; ++pair) {
            const int i = pair / p.sm.n, j = pair % p.sm.n;
            const int h = p.sm.h[j];
            const int y0 = (rb[i][0] - h) < 0 ? 0 : (rb[i][0] - h) / kSmTile;
            int y1 = (rb[i][1] + h) / kSmTile;
            if (y1 > ty - 1) y1 = ty - 1;
            const int xa0 = rb[i][2] / kSmTile, xa1 = rb[i][3] / kSmTile;
            const int xb0 = (rb[i][2] - h) < 0 ? 0 : (rb[i][2] - h) / kSmTile;
            int xb1 = (rb[i][3] + h) / kSmTile;
            if (xb1 > tx - 1) xb1 = tx - 1;
            const int ny = y1 - y0 + 1, nxa = xa1 - xa0 + 1, nxb = xb1 - xb0 + 1;
            // a tile joins a pass's list when its flag goes from 0 to 1
            for (int q = t; q < ny * nxa; q += blockDim.x) {
                const int64_t e = j * ntl + (int64_t)(y0 + q / nxa) * tx + xa0 + q % nxa;
                if (atomicExch(&p.sm.dirty_a[e], 1) == 0)
                    p.sm.list_a[atomicAdd(&p.sm.count[0], 1u)] = (int32_t)e;
            }
            for (int q = t; q < ny * nxb; q += blockDim.x) {
                const int64_t e = j * ntl + (int64_t)(y0 + q / nxb) * tx + xb0 + q % nxb;
                if (atomicExch(&p.sm.dirty_b[e], 1) == 0)
                    p.sm.list_b[atomicAdd(&p.sm.count[1], 1u)] = (int32_t)e;
            }
        }
    }
    if (st->pk.tiles_x > 0 && rank == 0) {
        // tiles of R that these windows touch, for the incremental peak search
        const PeakTiles K = st->pk;
        const int tx = K.tiles_x;
        for (int i = 0; i < nr; ++i) {
            const int y0 = rb[i][0] / kPkTile, y1 = rb[i][1] / kPkTile;
            const int x0 = rb[i][2] / kPkTile, x1 = rb[i][3] / kPkTile;
            const int nx = x1 - x0 + 1;
            for (int q = t; q < (y1 - y0 + 1) * nx; q += blockDim.x) {
                const int e = (y0 + q / nx) * tx + x0 + q % nx;
                if (atomicExch(&K.dirty[e], 1) == 0)
                    K.list[atomicAdd(K.count, 1u)] = e;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        dsq += __shfl_xor(dsq, off, 64);
    }
    if ((t & 63) == 0) {
        cnt_s[t >> 6] = cnt;
        dsq_s[t >> 6] = dsq;
    }
    __syncthreads();
    if (t == 0) {
        unsigned long long c = cnt_s[0] + cnt_s[1] + cnt_s[2] + cnt_s[3];
        if (c) {
            // the work-group's own slots of the pixel count and of the tracked
            // sum of R^2: the same work-group index in every launch, so no two
            // writers (no atomics on one counter from every work-group) and a
            // fixed order
            const int slot = rank % st->sq_nslots;
            st->px_slots[slot] += c;
            st->sq_slots[slot] += ((dsq_s[0] + dsq_s[1]) + dsq_s[2]) + dsq_s[3];
        }
    }
}

}  // namespace asp
