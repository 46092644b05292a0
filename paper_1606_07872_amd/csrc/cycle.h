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

// A streaming load: the scan reads each line once, so it is fetched with the
// non-temporal hint (measured: a 64 MiB scan from HBM-cold data in 16 us
// against 26 us with ordinary loads; no change when the data is cached).
typedef float f4v_t __attribute__((ext_vector_type(4)));
__device__ inline float4 load_stream(const float4 *p)
{
    const f4v_t v = __builtin_nontemporal_load(reinterpret_cast<const f4v_t *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
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
        float4 v0 = load_stream(R4 + i), v1 = load_stream(R4 + i + stride),
               v2 = load_stream(R4 + i + 2 * stride), v3 = load_stream(R4 + i + 3 * stride);
        peak_take4(v0, i, bv, bi);
        peak_take4(v1, i + stride, bv, bi);
        peak_take4(v2, i + 2 * stride, bv, bi);
        peak_take4(v3, i + 3 * stride, bv, bi);
    }
    for (; i < n4; i += stride) peak_take4(load_stream(R4 + i), i, bv, bi);
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
// Blocks stride over tiles of the plan's bounding box, 256 columns (origin a
// multiple of 4) by 4 kUpdPer rows, and skip tiles that meet no rect: a tile
// row is a 1 KiB run of memory (runs of 256 bytes measured 1.8x slower).  A
// circular Gaussian is separable, G(r, c) = a e^{-dy^2/2s^2} e^{-dx^2/2s^2}:
// per tile and rect the work-group tabulates the row factors (with the
// amplitude) and the 256 column factors in LDS, both zero outside the rect,
// so a pixel costs one FMA per rect and no exponential.  The tables hold
// kUpdChunk rects at a time (more rects take several passes over the same
// tile, adding in rect order), which keeps a work-group's LDS near 11 KiB:
// eight work-groups fit on a CU.  A thread takes four consecutive columns of
// kUpdPer rows (rows lr, lr + 4, ...): its float4 loads issued together, and
// float4 stores, when W is a multiple of 4.
// ===========================================================================

constexpr int kUpdCols = 256, kUpdRowStep = 4, kUpdRowsMax = 16, kUpdChunk = 8;
constexpr int kUpdTabFloats = kUpdChunk * (kUpdCols + kUpdRowsMax);   // factor tables in LDS

template <int kUpdPer = 4>
__device__ inline void update_tiles(const Params &p, int rank, int size, float *tab,
                                    bool need_ready = false)
{
    constexpr int kUpdRows = kUpdRowStep * kUpdPer;
    static_assert(kUpdRows <= kUpdRowsMax, "row tables");
    DevState *st = p.st;
    __shared__ int32_t rb[kMaxRects][4];
    __shared__ int32_t rcx[kMaxRects], rcy[kMaxRects];
    __shared__ float rfx[kMaxRects], rfy[kMaxRects], ramp[kMaxRects], rinv[kMaxRects];
    __shared__ uint32_t colbits[kUpdCols], rowbits[kUpdRowsMax];
    __shared__ int32_t nr_s, bb_s[4];
    __shared__ unsigned long long cnt_s[4];
    __shared__ double dsq_s[4];
    __shared__ double *sq_slot;
    __shared__ unsigned long long *px_slot;
    __shared__ PeakTiles pk_s;
    float *fx = tab;                               // [rect of the chunk][column of the tile]
    float *fy = tab + kUpdChunk * kUpdCols;        // [rect of the chunk][row], amplitude folded in
    const int t = threadIdx.x;
    __syncthreads();
    // the plan, read in one round trip: every rect slot is read, the unused
    // ones are never looked at
    if (t == 0) {
        const int32_t ready = need_ready ? st->fit_ready : 1;
        nr_s = ready ? st->n_rects : 0;
        for (int i = 0; i < 4; ++i) bb_s[i] = st->bb[i];
        // the work-group's own slots of the pixel count and of the tracked
        // sum of R^2: the same work-group index in every launch
        const int slot = rank % st->sq_nslots;
        sq_slot = st->sq_slots + slot;
        px_slot = st->px_slots + slot;
        pk_s = st->pk;
    }
    if (t < kMaxRects) {
        const Rect R = st->rects[t];
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
    const int32_t br0 = bb_s[0], br1 = bb_s[1], bc1 = bb_s[3];
    const int32_t bc0 = bb_s[2] & ~3;              // tiles start on a multiple of 4
    const int ntx = (bc1 - bc0 + kUpdCols) / kUpdCols, nty = (br1 - br0 + kUpdRows) / kUpdRows;
    // a bounding box lies inside the image (fewer than 2^32 pixels), so tile
    // indices fit in 32 bits
    const int32_t ntiles = nr > 0 ? ntx * nty : 0;
    static_assert(kMaxRects <= 32, "one bit per rect");
    static_assert(kUpdCols + kUpdRowsMax <= 2 * 256, "two masks per thread at most");
    const bool vec = (p.W & 3) == 0;
    uint32_t cnt32 = 0;
    double dsq = 0.0;                   // change of the sum of R^2 over this thread's pixels
    const int lr = t >> 6, lq = (t & 63) * 4;      // first row of the tile, first of 4 columns
    for (int32_t tile = rank; tile < ntiles; tile += size) {
        const int32_t ty = tile / ntx;
        const int32_t tr0 = br0 + ty * kUpdRows;
        const int32_t tc0 = bc0 + (tile - ty * ntx) * kUpdCols;
        bool any = false;
        for (int i = 0; i < nr; ++i)
            any |= (rb[i][0] <= tr0 + kUpdRows - 1 && tr0 <= rb[i][1] && rb[i][2] <= tc0 + kUpdCols - 1 &&
                    tc0 <= rb[i][3]);
        if (!any) continue;                        // the same for every thread
        const int32_t c = tc0 + lq;
        float v[kUpdPer][4];
        bool live[kUpdPer];
#pragma unroll
        for (int k = 0; k < kUpdPer; ++k) {
            const int32_t r = tr0 + lr + kUpdRowStep * k;
            live[k] = r <= br1 && c <= bc1;        // with vec, c .. c + 3 lie inside the image
            const int64_t q = (int64_t)r * p.W + c;
            v[k][0] = v[k][1] = v[k][2] = v[k][3] = 0.0f;
            if (live[k]) {
                if (vec) {
                    const float4 w = *reinterpret_cast<const float4 *>(p.R + q);
                    v[k][0] = w.x; v[k][1] = w.y; v[k][2] = w.z; v[k][3] = w.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (c + j < p.W) v[k][j] = p.R[q + j];
                }
            }
        }
        for (int e = t; e < kUpdCols + kUpdRows; e += blockDim.x) {
            uint32_t bits = 0u;
            if (e < kUpdCols) {
                const int32_t cc = tc0 + e;
                for (int i = 0; i < nr; ++i)
                    bits |= (cc >= rb[i][2] && cc <= rb[i][3]) ? (1u << i) : 0u;
                colbits[e] = bits;
            } else {
                const int32_t rr = tr0 + (e - kUpdCols);
                for (int i = 0; i < nr; ++i)
                    bits |= (rr >= rb[i][0] && rr <= rb[i][1]) ? (1u << i) : 0u;
                rowbits[e - kUpdCols] = bits;
            }
        }
        float acc[kUpdPer][4];
#pragma unroll
        for (int k = 0; k < kUpdPer; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[k][j] = 0.0f;
        for (int i0 = 0; i0 < nr; i0 += kUpdChunk) {
            const int nc = nr - i0 < kUpdChunk ? nr - i0 : kUpdChunk;
            if (i0 > 0) __syncthreads();           // the last chunk's tables are read
            // the factor tables of this chunk (the first while the loads above
            // are in flight)
            for (int e = t; e < nc * (kUpdCols + kUpdRows); e += blockDim.x) {
                const int ic = e / (kUpdCols + kUpdRows), j = e - ic * (kUpdCols + kUpdRows);
                const int i = i0 + ic;
                if (j < kUpdCols) {
                    const int32_t cc = tc0 + j;
                    const bool in = cc >= rb[i][2] && cc <= rb[i][3];
                    const float dx = (float)(cc - rcx[i]) - rfx[i];
                    fx[ic * kUpdCols + j] = in ? __expf(-(dx * dx) * rinv[i]) : 0.0f;
                } else {
                    const int32_t rr = tr0 + (j - kUpdCols);
                    const bool in = rr >= rb[i][0] && rr <= rb[i][1];
                    const float dy = (float)(rr - rcy[i]) - rfy[i];
                    fy[ic * kUpdRows + (j - kUpdCols)] =
                        in ? ramp[i] * __expf(-(dy * dy) * rinv[i]) : 0.0f;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kUpdPer; ++k) {
                for (int ic = 0; ic < nc; ++ic) {
                    const float gy = fy[ic * kUpdRows + lr + kUpdRowStep * k];
                    const float *gx = fx + ic * kUpdCols + lq;
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[k][j] += gy * gx[j];
                }
            }
        }
        uint32_t cb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) cb[j] = colbits[lq + j];
#pragma unroll
        for (int k = 0; k < kUpdPer; ++k) {
            if (live[k]) {
            const int32_t r = tr0 + lr + kUpdRowStep * k;
            const int64_t q = (int64_t)r * p.W + c;
            const uint32_t rbits = rowbits[lr + kUpdRowStep * k];
            bool hit[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) hit[j] = (rbits & cb[j]) != 0u;
            float nv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                nv[j] = hit[j] ? v[k][j] + acc[k][j] : v[k][j];
                if (hit[j]) {
                    dsq += (double)nv[j] * nv[j] - (double)v[k][j] * v[k][j];
                    ++cnt32;
                }
            }
            if (vec) {
                if (hit[0] || hit[1] || hit[2] || hit[3])
                    *reinterpret_cast<float4 *>(p.R + q) = make_float4(nv[0], nv[1], nv[2], nv[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (hit[j]) p.R[q + j] = nv[j];
            }
            }
        }
        __syncthreads();                           // the tables are rewritten by the next tile
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
    if (pk_s.tiles_x > 0 && rank == 0) {
        // tiles of R that these windows touch, for the incremental peak search
        const PeakTiles K = pk_s;
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
            // one writer per slot (no contention on one counter from every
            // work-group) and a fixed order; the adds return nothing, so the
            // work-group does not wait for a round trip on its way out
            atomicAdd(px_slot, c);
            unsafeAtomicAdd(sq_slot, ((dsq_s[0] + dsq_s[1]) + dsq_s[2]) + dsq_s[3]);
        }
    }
}

}  // namespace asp
