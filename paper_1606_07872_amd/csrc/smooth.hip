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
// rows (column pass) or h_j rows and columns (row pass) of its windows.
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

// Tiles of one scale in XCD-major order: work-group b runs on XCD b % 8 and
// takes the (b / 8)-th tile of that XCD's contiguous run, so that neighbours
// along the filter axis share their halos in one L2.
__device__ inline int xcd_tile(int b, int ntiles)
{
    const int per = (ntiles + 7) / 8;
    return (b % 8) * per + b / 8;
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

__global__ __launch_bounds__(kT) void k_smooth_cols(Params p, int force)
{
    if (!stale(p, force)) return;
    const int ntiles = p.sm.tiles_x * p.sm.tiles_y;
    const int j = blockIdx.y;
    // column-major tile order: consecutive tiles are vertical neighbours
    const int tile = xcd_tile(blockIdx.x, ntiles);
    if (tile >= ntiles) return;
    const int bx = tile / p.sm.tiles_y, by = tile % p.sm.tiles_y;
    const int id = by * p.sm.tiles_x + bx;
    int32_t *flag = p.sm.dirty_a + (int64_t)j * ntiles + id;
    if (*flag == 0) return;
    __shared__ float tr[TS][TS + 1];
    const int h = p.sm.h[j], nb = p.sm.nb[j];
    const int64_t lo = (int64_t)by * TS - h, hi = (int64_t)by * TS + (TS - RB) - h + RB * (nb + 1);
    if (lo >= 0 && hi <= p.H) cols_tile<false>(p, j, bx, by, tr);
    else cols_tile<true>(p, j, bx, by, tr);
    if (threadIdx.x == 0) *flag = 0;
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

__global__ __launch_bounds__(kT) void k_smooth_rows(Params p, int force)
{
    if (!stale(p, force)) return;
    const int ntiles = p.sm.tiles_x * p.sm.tiles_y;
    const int j = blockIdx.y;
    // row-major tile order: consecutive tiles are horizontal neighbours
    const int tile = xcd_tile(blockIdx.x, ntiles);
    if (tile >= ntiles) return;
    const int by = tile / p.sm.tiles_x, bx = tile % p.sm.tiles_x;
    int32_t *flag = p.sm.dirty_b + (int64_t)j * ntiles + tile;
    if (force < 2 && *flag == 0) return;
    const int h = p.sm.h[j], nb = p.sm.nb[j];
    const int64_t lo = (int64_t)bx * TS - h, hi = (int64_t)bx * TS + (TS - RB) - h + RB * (nb + 1);
    const int64_t rows_hi = (int64_t)by * TS + TS;
    unsigned long long best = (lo >= 0 && hi <= p.W && rows_hi <= p.H)
                                  ? rows_tile<false>(p, j, bx, by)
                                  : rows_tile<true>(p, j, bx, by);
    best = wave_max_key(best);
    __shared__ unsigned long long wk[kT / 64];
    if ((threadIdx.x & 63) == 0) wk[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = wk[0];
        for (int i = 1; i < kT / 64; ++i) m = wk[i] > m ? wk[i] : m;
        p.sm.keys[(int64_t)j * ntiles + tile] = m;
        *flag = 0;
    }
}

__device__ inline double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kT / 64; ++i) s += red[i];
    return s;
}

// The peak over the tile maxima, and the start values in FP64: the
// least-squares amplitude C / N of that scale's Gaussian on its window.
__global__ __launch_bounds__(kT) void k_smooth_pick(Params p, int force)
{
    if (!stale(p, force)) return;
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int64_t nk = (int64_t)p.sm.n * p.sm.tiles_x * p.sm.tiles_y;
    unsigned long long best = 0;
    for (int64_t i = t; i < nk; i += kT) {
        const unsigned long long k = p.sm.keys[i];
        best = k > best ? k : best;
    }
    best = wave_max_key(best);
    __shared__ unsigned long long wk[kT / 64];
    __shared__ double red[kT / 64];
    constexpr int kChunk = 1024;
    __shared__ double ey[kChunk];
    if ((t & 63) == 0) wk[t >> 6] = best;
    __syncthreads();
    best = wk[0];
    for (int i = 1; i < kT / 64; ++i) best = wk[i] > best ? wk[i] : best;
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
    // the window in chunks of kChunk rows; the row factors of a chunk in LDS,
    // thread t takes columns c0 + t, c0 + t + 256, ...
    double cs = 0.0, ns = 0.0;
    for (int64_t rb = r0; rb <= r1; rb += kChunk) {
        const int64_t re = rb + kChunk - 1 < r1 ? rb + kChunk - 1 : r1;
        __syncthreads();
        for (int64_t d = t; d <= re - rb; d += kT) {
            const double dd = (double)(rb + d - r);
            ey[d] = exp(-(dd * dd) * inv);
        }
        __syncthreads();
        for (int64_t cc = c0 + t; cc <= c1; cc += kT) {
            const double dx = (double)(cc - c);
            const double ex = exp(-(dx * dx) * inv);
            for (int64_t rr = rb; rr <= re; ++rr) {
                const double kv = ex * ey[rr - rb];
                cs += kv * (double)p.R[rr * W + cc];
                ns += kv * kv;
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

hipError_t launch_smooth(const Params &p, int force, hipStream_t s)
{
    const int ntiles = p.sm.tiles_x * p.sm.tiles_y;
    const dim3 grid((unsigned)(8 * ((ntiles + 7) / 8)), (unsigned)p.sm.n);
    hipLaunchKernelGGL(k_smooth_cols, grid, dim3(kT), 0, s, p, force);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_rows, grid, dim3(kT), 0, s, p, force);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_pick, dim3(1), dim3(kT), 0, s, p, force);
    return hipGetLastError();
}

}  // namespace asp
