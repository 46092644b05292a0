// Incremental peak search (Sect. 2 step 1): the largest |R|, the lowest
// row-major index winning ties, from per-tile maxima kept on the device.
//
// A residual update changes R only inside its windows, so only the 64 x 64
// tiles those windows touch can change their maximum.  The update lists each
// such tile once (its stale flag going from 0 to 1); here a fixed grid rescans
// the listed tiles, and one work-group reduces all tile keys into the peak
// key.  The packed key (|v| bits << 32) | (0xFFFFFFFF - idx) is the one of the
// full scan, so the result is the same pixel bit for bit.
#include "asp_device.h"

namespace asp {
namespace {

constexpr int kT = 256;
constexpr int kReduceT = 1024;
constexpr int kTileGrid = 1024;

__device__ inline unsigned long long wave_max(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Lane = column of the tile, wave w = rows w, w + 4, ...: every load of a wave
// is one 256-byte row segment.
__global__ __launch_bounds__(kT) void k_peak_tiles(Params p)
{
    if (p.st->stop) return;
    const PeakTiles K = p.st->pk;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int tx = K.tiles_x;
    const unsigned int n = K.count[0];
    const int64_t H = p.H, W = p.W;
    __shared__ unsigned long long wk[kT / 64];
    for (unsigned int i = blockIdx.x; i < n; i += gridDim.x) {
        const int tile = K.list[i];
        const int64_t r0 = (int64_t)(tile / tx) * kPkTile;
        const int64_t c = (int64_t)(tile % tx) * kPkTile + lane;
        unsigned long long best = 0;
        if (c < W) {
            // rows in increasing order, strict maximum: the lowest index of a tie
            float bv = -1.0f;
            int64_t bi = 0;
            for (int rr = w; rr < kPkTile; rr += kT / 64) {
                const int64_t r = r0 + rr;
                if (r >= H) break;
                const float a = fabsf(p.R[r * W + c]);
                if (a > bv) { bv = a; bi = r * W + c; }
            }
            if (bv >= 0.0f)
                best = ((unsigned long long)__float_as_uint(bv) << 32) |
                       (unsigned long long)(0xFFFFFFFFu - (uint32_t)bi);
        }
        best = wave_max(best);
        __syncthreads();                   // wk of the previous tile is read
        if (lane == 0) wk[w] = best;
        __syncthreads();
        if (t == 0) {
            unsigned long long m = wk[0];
            for (int k = 1; k < kT / 64; ++k) m = wk[k] > m ? wk[k] : m;
            K.keys[tile] = m;
            K.dirty[tile] = 0;
            atomicAdd(&p.st->pk_tiles_done, 1ull);
        }
    }
}

// The maximum of the tile keys into the peak key (slot 0; the slots are
// cleared by whoever consumes the key).  The tile pass has finished: its list
// is emptied here.
__global__ __launch_bounds__(kReduceT) void k_peak_reduce(Params p)
{
    if (p.st->stop) return;
    const PeakTiles K = p.st->pk;
    const int t = threadIdx.x;
    if (t == 0) K.count[0] = 0;
    const int ntiles = K.tiles_x * K.tiles_y;
    unsigned long long best = 0;
    for (int i = t; i < ntiles; i += kReduceT) {
        const unsigned long long k = K.keys[i];
        best = k > best ? k : best;
    }
    best = wave_max(best);
    __shared__ unsigned long long wk[kReduceT / 64];
    if ((t & 63) == 0) wk[t >> 6] = best;
    __syncthreads();
    if (t == 0) {
        unsigned long long m = wk[0];
        for (int k = 1; k < kReduceT / 64; ++k) m = wk[k] > m ? wk[k] : m;
        atomicMax(&p.st->peak_keys[0], m);
    }
}

__global__ __launch_bounds__(kT) void k_peak_mark_all(Params p)
{
    const PeakTiles K = p.st->pk;
    const int ntiles = K.tiles_x * K.tiles_y;
    for (int i = blockIdx.x * kT + threadIdx.x; i < ntiles; i += gridDim.x * kT) {
        K.dirty[i] = 1;
        K.list[i] = i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) K.count[0] = (unsigned int)ntiles;
}

}  // namespace

hipError_t launch_peak_tiles(const Params &p, int ntiles, hipStream_t s)
{
    const int grid = ntiles < kTileGrid ? ntiles : kTileGrid;
    hipLaunchKernelGGL(k_peak_tiles, dim3(grid), dim3(kT), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_peak_reduce, dim3(1), dim3(kReduceT), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_peak_mark_all(const Params &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_peak_mark_all, dim3(64), dim3(kT), 0, s, p);
    return hipGetLastError();
}

}  // namespace asp
