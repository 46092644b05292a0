// The smoothing method of initial values (Sect. 2 step 1; Sect. 3): the
// residual smoothed with Gaussian beams of a few widths, and the peak over all
// smoothed images.
//
// The 2-D window sum of a Gaussian beam factors into a column pass and a row
// pass, each a 1-D filter of 2h + 1 taps.  The column pass V_j = k_j (*)cols R
// is kept on the device for every trial width (transposed, W x H, so that the
// row pass reads it with unit stride); the row pass gives C_j and its maxima
// per 64 x 64 tile and scale.  Only tiles whose inputs a residual update
// changed are recomputed: the update marks, per scale, the tiles within h_j
// rows (column pass) or h_j rows and columns (row pass) of its windows, and
// appends each newly stale (scale, tile) to the pass's list; a fixed grid of
// work-groups walks the lists.
//
// Each pass is a register-blocked FIR: a thread owns kSmRb consecutive
// outputs along the filter axis, the 64 lanes of a wave own 64 neighbouring
// lines, so that every load of a wave is one contiguous 256-byte row, and the
// taps are uniform (scalar) operands of the FMAs.  No LDS is needed except to
// transpose the column pass on its way out.
#include "asp_device.h"

namespace asp {
namespace {

constexpr int kT = 256;
constexpr int TS = kSmTile;
constexpr int RB = kSmRb;
constexpr int kPassGrid = 2048;     // work-groups of a pass: 8 per compute unit (a multiple of 8)

// out[i] = sum_{d < RB nb} k[d] x(i + d), i < RB, accumulated in order of d;
// x(e) is read for e < RB (nb + 1).
template <typename Load>
__device__ __forceinline__ void fir(const float *__restrict__ k, int nb, Load load,
                                    float (&out)[RB])
{
    float cur[RB], nxt[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        out[i] = 0.0f;
        cur[i] = load(i);
    }
    for (int b = 0; b < nb; ++b) {
#pragma unroll
        for (int i = 0; i < RB; ++i) nxt[i] = load((b + 1) * RB + i);
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const float kk = k[b * RB + u];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const float xv = (u + i < RB) ? cur[u + i] : nxt[u + i - RB];
                out[i] = fmaf(kk, xv, out[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) cur[i] = nxt[i];
    }
}

// Entries of a list in XCD-contiguous chunks: work-group b runs on XCD b % 8
// and takes the entries lo + b / 8, lo + b / 8 + G / 8, ... of that XCD's
// eighth of the list, so that neighbouring tiles (consecutive entries), whose
// halos overlap, are read through one L2.
struct Chunk {
    unsigned int i, hi, step;
};

__device__ inline Chunk xcd_chunk(unsigned int n)
{
    const unsigned int per = (n + 7) / 8, x = blockIdx.x % 8;
    const unsigned int lo = x * per;
    return {lo + blockIdx.x / 8, lo + per < n ? lo + per : n, gridDim.x / 8};
}

__device__ inline bool stale(const Params &p, int force)
{
    const DevState *st = p.st;
    if (force) return true;
    return st->stop == 0 && st->smooth_now != 0;
}

// Column pass of one (tile, scale): V_j(r, c) = sum_{|d| <= h} k(d) R(r + d, c),
// R = 0 outside the image; stored as vt[j][c][r].
template <bool kCheck>
__device__ __forceinline__ void cols_tile(const Params &p, int j, int bx, int by,
                                          float (*tr)[TS + 1])
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t H = p.H, W = p.W;
    const int h = p.sm.h[j], nb = p.sm.nb[j];
    const float *k = p.sm.taps + p.sm.off[j];
    const int64_t c = (int64_t)bx * TS + lane;
    const int64_t r0 = (int64_t)by * TS + w * RB - h;     // row of x(0)
    const bool col_ok = c < W;
    const float *Rc = p.R + (col_ok ? c : 0);
    float out[RB];
    fir(k, nb,
        [&](int e) -> float {
            const int64_t r = r0 + e;
            if (kCheck) return (col_ok && r >= 0 && r < H) ? Rc[r * W] : 0.0f;
            return Rc[r * W];
        },
        out);
#pragma unroll
    for (int i = 0; i < RB; ++i) tr[lane][w * RB + i] = out[i];
    __syncthreads();
    float *vt = p.sm.vt + (int64_t)j * H * W;
    const int64_t rr = (int64_t)by * TS + lane;
    for (int q = 0; q < RB; ++q) {
        const int cl = w * RB + q;
        const int64_t cc = (int64_t)bx * TS + cl;
        if (cc < W && rr < H) vt[cc * H + rr] = tr[cl][lane];
    }
}

// The column pass over its list of stale (scale, tile) entries.
__global__ __launch_bounds__(kT) void k_smooth_cols(Params p, int force)
{
    if (!stale(p, force)) return;
    const int tx = p.sm.tiles_x, ntiles = tx * p.sm.tiles_y;
    const Chunk ch = xcd_chunk(p.sm.count[0]);
    __shared__ float tr[TS][TS + 1];
    for (unsigned int i = ch.i; i < ch.hi; i += ch.step) {
        const int e = p.sm.list_a[i];
        const int j = e / ntiles, tile = e % ntiles;
        const int by = tile / tx, bx = tile % tx;
        const int h = p.sm.h[j], nb = p.sm.nb[j];
        const int64_t lo = (int64_t)by * TS - h;
        const int64_t hi = (int64_t)by * TS + (TS - RB) - h + RB * (nb + 1);
        __syncthreads();                   // tr of the previous entry is read
        if (lo >= 0 && hi <= p.H) cols_tile<false>(p, j, bx, by, tr);
        else cols_tile<true>(p, j, bx, by, tr);
        if (threadIdx.x == 0) {
            p.sm.dirty_a[e] = 0;
            const int64_t rows = p.H - (int64_t)by * TS < TS ? p.H - (int64_t)by * TS : TS;
            const int64_t cols = p.W - (int64_t)bx * TS < TS ? p.W - (int64_t)bx * TS : TS;
            atomicAdd(&p.st->sm_px[j], (unsigned long long)(rows * cols));
        }
    }
}

// Row pass of one (tile, scale): C_j(r, c) = sum_{|d| <= h} k(d) V_j(r, c + d),
// V = 0 outside the image; the tile's packed maximum of the score
// (|score| bits << 32 | 0xFFFFFFFF - (j N + p)) goes to keys[j][tile].
template <bool kCheck>
__device__ __forceinline__ unsigned long long rows_tile(const Params &p, int j, int bx, int by)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t H = p.H, W = p.W, N = H * W;
    const int h = p.sm.h[j], nb = p.sm.nb[j];
    const float *k = p.sm.taps + p.sm.off[j];
    const int64_t r = (int64_t)by * TS + lane;
    const int64_t cb = (int64_t)bx * TS + w * RB;        // first output column
    const int64_t c0 = cb - h;                           // column of x(0)
    const bool row_ok = r < H;
    const float *V = p.sm.vt + (int64_t)j * N + (row_ok ? r : 0);
    float out[RB];
    fir(k, nb,
        [&](int e) -> float {
            const int64_t cc = c0 + e;
            if (kCheck) return (row_ok && cc >= 0 && cc < W) ? V[cc * H] : 0.0f;
            return V[cc * H];
        },
        out);
    unsigned long long best = 0;
    if (row_ok) {
        const float wy = p.sm.norm ? p.sm.wy[(int64_t)j * H + r] : 1.0f;
        const bool want_map = p.sm.map && p.sm.map_scale == j;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int64_t cc = cb + i;
            if (cc >= W) break;
            float v = out[i];
            if (p.sm.norm) v = v * (p.sm.wx[(int64_t)j * W + cc] * wy);
            if (want_map) p.sm.map[r * W + cc] = v;
            const uint32_t q = (uint32_t)((int64_t)j * N + r * W + cc);
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(fabsf(v)) << 32) |
                (unsigned long long)(0xFFFFFFFFu - q);
            best = key > best ? key : best;
        }
    }
    return best;
}

__device__ inline unsigned long long wave_max_key(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// The row pass over its list of stale (scale, tile) entries (every entry with
// force 2).  The column pass has finished: its list is emptied here.
__global__ __launch_bounds__(kT) void k_smooth_rows(Params p, int force)
{
    if (!stale(p, force)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) p.sm.count[0] = 0;
    const int tx = p.sm.tiles_x, ntiles = tx * p.sm.tiles_y;
    const Chunk ch = xcd_chunk(force == 2 ? (unsigned int)(p.sm.n * ntiles) : p.sm.count[1]);
    __shared__ unsigned long long wk[kT / 64];
    for (unsigned int i = ch.i; i < ch.hi; i += ch.step) {
        const int e = force == 2 ? (int)i : p.sm.list_b[i];
        const int j = e / ntiles, tile = e % ntiles;
        const int by = tile / tx, bx = tile % tx;
        const int h = p.sm.h[j], nb = p.sm.nb[j];
        const int64_t lo = (int64_t)bx * TS - h;
        const int64_t hi = (int64_t)bx * TS + (TS - RB) - h + RB * (nb + 1);
        const int64_t rows_hi = (int64_t)by * TS + TS;
        unsigned long long best = (lo >= 0 && hi <= p.W && rows_hi <= p.H)
                                      ? rows_tile<false>(p, j, bx, by)
                                      : rows_tile<true>(p, j, bx, by);
        best = wave_max_key(best);
        __syncthreads();                   // wk of the previous entry is read
        if ((threadIdx.x & 63) == 0) wk[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long m = wk[0];
            for (int k = 1; k < kT / 64; ++k) m = wk[k] > m ? wk[k] : m;
            p.sm.keys[e] = m;
            p.sm.dirty_b[e] = 0;
            const int64_t rows = p.H - (int64_t)by * TS < TS ? p.H - (int64_t)by * TS : TS;
            const int64_t cols = p.W - (int64_t)bx * TS < TS ? p.W - (int64_t)bx * TS : TS;
            atomicAdd(&p.st->sm_px[kMaxScales + j], (unsigned long long)(rows * cols));
        }
    }
}

// Every entry stale.  The lists hold the tiles in row-major order with the
// scales of a tile side by side, so that an XCD's chunk is a band of tiles
// with all their scales (the cost of a tile grows with its scale).
__global__ __launch_bounds__(kT) void k_smooth_mark_all(Params p)
{
    const int64_t ntiles = (int64_t)p.sm.tiles_x * p.sm.tiles_y;
    const int64_t n = (int64_t)p.sm.n * ntiles;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        p.sm.dirty_a[i] = 1;
        p.sm.dirty_b[i] = 1;
        const int32_t e = (int32_t)((i % p.sm.n) * ntiles + i / p.sm.n);
        p.sm.list_a[i] = e;
        p.sm.list_b[i] = e;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.sm.count[0] = (unsigned int)n;
        p.sm.count[1] = (unsigned int)n;
    }
}

constexpr int kPickT = 1024;        // threads of the pick: 16 waves
constexpr int kPickChunk = 2048;    // window rows (columns) per LDS table

__device__ inline double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kPickT / 64; ++i) s += red[i];
    return s;
}

// The peak over the tile maxima, and the start values in FP64: the
// least-squares amplitude C / N of that scale's Gaussian on its window.  The
// window's row and column factors exp(-d^2 / (2 sigma^2)) go to LDS; wave w
// sums rows w, w + 16, ..., its lanes 64 consecutive columns at a time.
__global__ __launch_bounds__(kPickT) void k_smooth_pick(Params p, int force)
{
    if (!stale(p, force)) return;
    DevState *st = p.st;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) p.sm.count[1] = 0;        // the row pass has finished its list
    const int64_t nk = (int64_t)p.sm.n * p.sm.tiles_x * p.sm.tiles_y;
    unsigned long long best = 0;
    for (int64_t i = t; i < nk; i += kPickT) {
        const unsigned long long k = p.sm.keys[i];
        best = k > best ? k : best;
    }
    best = wave_max_key(best);
    __shared__ unsigned long long wk[kPickT / 64];
    __shared__ double red[kPickT / 64];
    __shared__ double ex[kPickChunk], ey[kPickChunk];
    if (lane == 0) wk[w] = best;
    __syncthreads();
    best = wk[0];
    for (int i = 1; i < kPickT / 64; ++i) best = wk[i] > best ? wk[i] : best;
    const int64_t H = p.H, W = p.W, N = H * W;
    const uint32_t q = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
    const int j = (int)(q / (uint64_t)N);
    if (best == 0ull || j >= p.sm.n) {
        if (t == 0) { st->smooth_ready = 0; st->stop = ASP_ERR_DEVICE; }
        return;
    }
    const int64_t pix = (int64_t)q - (int64_t)j * N;
    const int64_t r = pix / W, c = pix % W;
    const double sig = p.sm.sig[j];
    const double inv = 1.0 / (2.0 * sig * sig);
    const int64_t h = p.sm.h[j];
    const int64_t r0 = r - h > 0 ? r - h : 0, r1 = r + h < H - 1 ? r + h : H - 1;
    const int64_t c0 = c - h > 0 ? c - h : 0, c1 = c + h < W - 1 ? c + h : W - 1;
    double cs = 0.0, ns = 0.0;
    for (int64_t rb = r0; rb <= r1; rb += kPickChunk) {
        const int64_t re = rb + kPickChunk - 1 < r1 ? rb + kPickChunk - 1 : r1;
        for (int64_t cb = c0; cb <= c1; cb += kPickChunk) {
            const int64_t ce = cb + kPickChunk - 1 < c1 ? cb + kPickChunk - 1 : c1;
            __syncthreads();
            for (int64_t d = t; d <= re - rb; d += kPickT) {
                const double dd = (double)(rb + d - r);
                ey[d] = exp(-(dd * dd) * inv);
            }
            for (int64_t d = t; d <= ce - cb; d += kPickT) {
                const double dd = (double)(cb + d - c);
                ex[d] = exp(-(dd * dd) * inv);
            }
            __syncthreads();
            const int nr = (int)(re - rb + 1), nc = (int)(ce - cb + 1);
            for (int rr = w; rr < nr; rr += kPickT / 64) {
                const double fy = ey[rr];
                const float *row = p.R + (rb + rr) * W + cb;
#pragma unroll 4
                for (int cc = lane; cc < nc; cc += 64) {
                    const double kv = ex[cc] * fy;
                    cs += kv * (double)row[cc];
                    ns += kv * kv;
                }
            }
        }
    }
    cs = block_sum(cs, red);
    ns = block_sum(ns, red);
    if (t == 0) {
        st->smooth_start[0] = cs / ns;
        st->smooth_start[1] = (double)c;
        st->smooth_start[2] = (double)r;
        st->smooth_start[3] = sig;
        st->smooth_scale = j;
        st->smooth_idx = pix;
        st->smooth_score = __uint_as_float((uint32_t)(best >> 32));
        st->smooth_ready = 1;
    }
}

}  // namespace

hipError_t launch_smooth_passes(const Params &p, int force, hipStream_t s)
{
    const int64_t entries = (int64_t)p.sm.n * p.sm.tiles_x * p.sm.tiles_y;
    const int64_t g = entries < kPassGrid ? entries : kPassGrid;
    const unsigned grid = (unsigned)(8 * ((g + 7) / 8));      // a multiple of the 8 XCDs
    hipLaunchKernelGGL(k_smooth_cols, dim3(grid), dim3(kT), 0, s, p, force);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_rows, dim3(grid), dim3(kT), 0, s, p, force);
    return hipGetLastError();
}

hipError_t launch_smooth_mark_all(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_smooth_mark_all, dim3(256), dim3(kT), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_smooth_pick(const Params &p, int force, hipStream_t s)
{
    hipLaunchKernelGGL(k_smooth_pick, dim3(1), dim3(kPickT), 0, s, p, force);
    return hipGetLastError();
}

}  // namespace asp
