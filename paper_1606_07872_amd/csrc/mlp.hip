// The learned start-value proposal: a 1024-256-256-4 perceptron that maps
// the residual patch around the peak to the start point of the new
// component's fit, in place of the simple initial values of Sect. 3 (the
// residual peak and the main-lobe width).  The LM fit of Sect. 3 runs from the
// proposal and decides whether it is kept: when that fit does not converge,
// or ends with a new component of amplitude zero, the fit kernel fits the
// simple values instead.
//
// Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3.
//   x = the 32 x 32 patch around the peak pixel (r*, c*), rows r*-16..r*+15,
//       columns c*-16..c*+15, zero outside the image, divided by R[p*];
//   y = (a / R[p*], log(s / omega_b), x - c*, y - r*) of the fitted new
//       component (convolved space, before the loop gain).
// Flat parameter order: W1 (256 x 1024, row-major), b1, W2 (256 x 256), b2,
// W3 (4 x 256), b3; 329220 FP32 values.
//
// This file holds
//   * the inference kernel of the minor cycle (64 work-groups, which also
//     record the patch of (patch, target) training pairs when asked),
//   * the training kernels: a tiled FP32 GEMM with fused bias / ReLU / ReLU
//     mask epilogues, column sums, the MSE gradient, Adam and a row gather,
//   * the trainer object of the C ABI (asp_mlp_*).
// The training loss is the mean over samples and outputs of (y - t)^2.
#include <math.h>
#include <string.h>

#include <string>

#include "asp_device.h"

namespace asp {

// ===========================================================================
// Inference inside the minor cycle.
// ===========================================================================

constexpr int kPT = 256;                          // threads per work-group
constexpr int kUnits = kNetH / kPropGroups;       // first-layer units per work-group
constexpr int kPerThread = kNetIn / kPT;          // patch inputs per thread
static_assert(kNetH == kPT, "one thread per second-layer unit");
static_assert(kNetOut * 64 == kPT, "one wave per output");
static_assert(kUnits * kPropGroups == kNetH && kUnits == 4, "four first-layer units per group");
static_assert(kPerThread == 4 && kPatch % kPerThread == 0, "four inputs of one patch row");

// The peak pixel of this iteration (the forced index of a caller's fit, else
// the decoded peak key) and the residual there; false when there is none (the
// fit kernel reports that state) or after a stop.  The stop flag, the forced
// index and the key slots are read in one round trip.  Every thread of the
// work-group calls it.
__device__ inline bool proposal_centre(const Params &p, unsigned long long *key_s, int64_t *r0,
                                       int64_t *c0, float *v)
{
    DevState *st = p.st;
    const int32_t stop = st->stop;
    int64_t idx = st->forced_idx;
    const unsigned long long key = collect_peak_key(st, false, key_s);
    if (stop) return false;
    if (idx < 0) {
        if (key == 0ull) return false;
        idx = (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    }
    if (idx >= p.H * p.W) return false;
    *r0 = idx / p.W;
    *c0 = idx % p.W;
    *v = p.R[idx];
    return true;
}

// One launch of kPropGroups work-groups.  Work-group g:
//   * gathers the whole patch (thread t holds inputs 4t .. 4t+3, four
//     neighbours of one patch row) and, when the context collects training
//     pairs, records inputs 16g .. 16g+15;
//   * forms first-layer units 4g .. 4g+3 completely (per-thread products,
//     then a fixed-order reduction over lanes and waves);
//   * writes the contribution of those four units to every second-layer
//     pre-activation (thread u: unit u), one row of the partial-sum scratch.
// The work-group that arrives last adds the rows in work-group order, applies
// the bias and ReLU, runs the output layer and writes the proposal.  Every
// load that does not depend on another is issued at the start.  Without a
// peak, or after a stop, every work-group leaves before the arrival, so the
// counter stays a multiple of the grid.
__global__ __launch_bounds__(kPT) void k_propose(Params p, NetParams net, int use_net)
{
    DevState *st = p.st;
    __shared__ float red[kPT / 64][kUnits];
    __shared__ float h1[kUnits];
    __shared__ float h2[kNetH];
    __shared__ float outs[kNetOut];
    __shared__ unsigned long long key_s;
    __shared__ int last_s;
    const int t = threadIdx.x, g = blockIdx.x;
    const int wave = t >> 6, lane = t & 63;
    float4 w1[kUnits];
    float w2[kUnits], w3[kNetH / 64];
    float b1 = 0.0f, b2 = 0.0f, b3 = 0.0f;
    if (use_net) {
#pragma unroll
        for (int j = 0; j < kUnits; ++j)
            w1[j] = *reinterpret_cast<const float4 *>(net.w1 + (int64_t)(g * kUnits + j) * kNetIn +
                                                      kPerThread * t);
#pragma unroll
        for (int j = 0; j < kUnits; ++j) w2[j] = net.w2t[(g * kUnits + j) * kNetH + t];
#pragma unroll
        for (int i = 0; i < kNetH / 64; ++i) w3[i] = net.w3[wave * kNetH + lane + 64 * i];
        b1 = t < kUnits ? net.b1[g * kUnits + t] : 0.0f;
        b2 = net.b2[t];
        b3 = lane == 0 ? net.b3[wave] : 0.0f;
    }
    int64_t r0, c0;
    float v;
    if (!proposal_centre(p, &key_s, &r0, &c0, &v)) return;
    float x[kPerThread];
    {
        const int e0 = kPerThread * t;
        const int64_t r = r0 - kPatchHalf + e0 / kPatch;
        const int64_t cb = c0 - kPatchHalf + e0 % kPatch;
        const bool row_in = r >= 0 && r < p.H;
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            const int64_t c = cb + i;
            x[i] = (row_in && c >= 0 && c < p.W) ? p.R[r * p.W + c] / v : 0.0f;
        }
        if (p.rec_cap > 0 && (e0 >> 4) == g && st->rec_n < p.rec_cap) {
            float *rp = p.rec_patch + st->rec_n * kNetIn + e0;
#pragma unroll
            for (int i = 0; i < kPerThread; ++i) rp[i] = x[i];
        }
    }
    if (!use_net) return;
    // first layer: units 4g .. 4g+3
    {
        float acc[kUnits];
#pragma unroll
        for (int j = 0; j < kUnits; ++j)
            acc[j] = w1[j].x * x[0] + w1[j].y * x[1] + w1[j].z * x[2] + w1[j].w * x[3];
#pragma unroll
        for (int j = 0; j < kUnits; ++j)
            for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
        if (lane < kUnits) {
            float a = acc[0];
#pragma unroll
            for (int j = 1; j < kUnits; ++j) a = lane == j ? acc[j] : a;
            red[wave][lane] = a;
        }
        __syncthreads();
        if (t < kUnits) {
            float a = b1;
#pragma unroll
            for (int q = 0; q < kPT / 64; ++q) a += red[q][t];
            h1[t] = a > 0.0f ? a : 0.0f;
        }
        __syncthreads();
    }
    // this group's share of every second-layer pre-activation
    {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < kUnits; ++j) a += w2[j] * h1[j];
        net.part[g * kNetH + t] = a;
    }
    // arrival: the barrier orders every thread's stores before thread 0's
    // release; the last arrival's acquire pairs with the others' releases
    __syncthreads();
    if (t == 0) {
        const unsigned int before = __hip_atomic_fetch_add(net.done, 1u, __ATOMIC_ACQ_REL,
                                                           __HIP_MEMORY_SCOPE_AGENT);
        last_s = (before + 1u) % kPropGroups == 0u ? 1 : 0;
    }
    __syncthreads();
    if (!last_s) return;
    {
        float part[kPropGroups];
#pragma unroll
        for (int q = 0; q < kPropGroups; ++q)
            part[q] = __hip_atomic_load(&net.part[q * kNetH + t], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        float a = b2;
#pragma unroll
        for (int q = 0; q < kPropGroups; ++q) a += part[q];
        h2[t] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < kNetH / 64; ++i) a += w3[i] * h2[lane + 64 * i];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == 0) outs[wave] = a + b3;
    }
    __syncthreads();
    if (t == 0) {
        const double vv = (double)v;
        st->proposal[0] = (double)outs[0] * vv;
        st->proposal[1] = (double)c0 + (double)outs[2];
        st->proposal[2] = (double)r0 + (double)outs[3];
        st->proposal[3] = st->omega_b * exp((double)outs[1]);
        st->have_proposal = 2;
    }
}

hipError_t launch_propose(const Params &p, const NetParams &net, int use_net, hipStream_t s)
{
    hipLaunchKernelGGL(k_propose, dim3(kPropGroups), dim3(kPT), 0, s, p, net, use_net);
    return hipGetLastError();
}

// ===========================================================================
// Training kernels.
// ===========================================================================

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn], then the epilogue:
//   kEpiPlain    C
//   kEpiBias     C + bias[n]
//   kEpiBiasRelu max(C + bias[n], 0)
//   kEpiMask     C where mask[m ldc + n] > 0, else 0 (the ReLU derivative)
enum { kEpiPlain = 0, kEpiBias = 1, kEpiBiasRelu = 2, kEpiMask = 3 };

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    float *C;
    int64_t ldc;
    const float *bias, *mask;
    int epi;
};

constexpr int kBM = 64, kBN = 64, kBK = 16;

// 64 x 64 output tile per 256-thread work-group, 4 x 4 per thread, K in steps
// of 16 through LDS.  Each operand tile is loaded with the thread order that
// makes its unit-stride dimension the fast one.  The k order of the sums is
// fixed, so results are deterministic.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ float As[kBK][kBM + 4];
    __shared__ float Bs[kBK][kBN + 4];
    const int t = threadIdx.x;
    const int tm = t / 16, tn = t % 16;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    float acc[4][4] = {};
    const bool a_m_fast = g.sam == 1 && g.sak != 1;
    const bool b_k_fast = g.sbk == 1 && g.sbn != 1;
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = t + 256 * i;
            int row, kk;
            if (a_m_fast) { row = e % kBM; kk = e / kBM; }
            else { row = e / kBK; kk = e % kBK; }
            const int m = m0 + row, k = k0 + kk;
            As[kk][row] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = t + 256 * i;
            int col, kk;
            if (b_k_fast) { col = e / kBK; kk = e % kBK; }
            else { col = e % kBN; kk = e / kBN; }
            const int n = n0 + col, k = k0 + kk;
            Bs[kk][col] = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kBK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tm * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + tm * 4 + i;
        if (m >= g.M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tn * 4 + j;
            if (n >= g.N) continue;
            float v = acc[i][j];
            const int64_t o = (int64_t)m * g.ldc + n;
            if (g.epi == kEpiBias || g.epi == kEpiBiasRelu) v += g.bias[n];
            if (g.epi == kEpiBiasRelu) v = v > 0.0f ? v : 0.0f;
            if (g.epi == kEpiMask) v = g.mask[o] > 0.0f ? v : 0.0f;
            g.C[o] = v;
        }
    }
}

// out[n] = sum over m of X[m ld + n], in row order (the bias gradients).
__global__ void k_colsum(const float *X, int M, int N, int64_t ld, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int m = 0; m < M; ++m) s += X[(int64_t)m * ld + n];
    out[n] = s;
}

// dY = 2 (Y - T) / (B d) and the batch loss sum((Y - T)^2) / (B d), one
// work-group, fixed summation order.
__global__ __launch_bounds__(256) void k_mse(const float *Y, const float *T, int n, float *dY,
                                             double *loss)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0.0;
    const float scale = 2.0f / (float)n;
    for (int i = t; i < n; i += 256) {
        const float d = Y[i] - T[i];
        dY[i] = scale * d;
        s += (double)d * (double)d;
    }
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) *loss += red[0] / (double)n;
}

// Adam (Kingma & Ba 2015); c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void k_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// dst[b][:] = src[idx[b]][:] for rows of `len` floats; an index outside
// [0, n_src) gives a zero row and sets *bad.
__global__ void k_gather(const float *src, int64_t n_src, const int32_t *idx, int rows, int len,
                         float *dst, int32_t *bad)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * len) return;
    const int b = (int)(e / len), j = (int)(e % len);
    const int64_t r = idx[b];
    if (r < 0 || r >= n_src) {
        dst[e] = 0.0f;
        if (j == 0) *bad = 1;
        return;
    }
    dst[e] = src[r * len + j];
}

// Input-major copy of W (rows x cols, row-major): wt[c][r] = w[r][c].
__global__ void k_transpose(const float *w, int rows, int cols, float *wt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    wt[(int64_t)c * rows + r] = w[e];
}

hipError_t launch_net_layout(const float *flat, float *net, hipStream_t s)
{
    // flat: W1 (256 x 1024), b1, W2 (256 x 256), b2, W3, b3
    // net:  W1, b1, W2^T (256 x 256), b2, W3, b3
    const int64_t n1 = (int64_t)kNetH * kNetIn, n2 = (int64_t)kNetH * kNetH;
    hipError_t e = hipMemcpyAsync(net, flat, sizeof(float) * (n1 + kNetH),
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                       flat + n1 + kNetH, kNetH, kNetH, net + n1 + kNetH);
    const int64_t tail = kNetParams - (n1 + kNetH + n2);
    return hipMemcpyAsync(net + n1 + kNetH + n2, flat + n1 + kNetH + n2, sizeof(float) * tail,
                          hipMemcpyDeviceToDevice, s);
}

}  // namespace asp

// ===========================================================================
// The trainer of the C ABI.
// ===========================================================================

using namespace asp;

struct asp_mlp {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int bmax = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // kNetParams each
    float *X = nullptr, *T = nullptr;                               // bmax x 1024, bmax x 4
    float *H1 = nullptr, *H2 = nullptr, *Y = nullptr;
    float *dY = nullptr, *dH1 = nullptr, *dH2 = nullptr;
    double *loss = nullptr;
    int32_t *bad = nullptr;                                         // gather index error
    int64_t t = 0;                                                  // Adam steps taken
    std::string err;
};

namespace {

constexpr int64_t kOffB1 = (int64_t)kNetH * kNetIn;
constexpr int64_t kOffW2 = kOffB1 + kNetH;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kNetH * kNetH;
constexpr int64_t kOffW3 = kOffB2 + kNetH;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kNetOut * kNetH;

asp_status mfail(asp_mlp *n, asp_status s, const std::string &msg)
{
    if (n) n->err = msg;
    return s;
}

#define MLP_HIP(n, call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return mfail((n), ASP_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

hipError_t gemm(hipStream_t s, int M, int N, int K, const float *A, int64_t sam, int64_t sak,
                const float *B, int64_t sbk, int64_t sbn, float *C, int64_t ldc, int epi,
                const float *bias = nullptr, const float *mask = nullptr)
{
    GemmArgs a{M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, mask, epi};
    dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t colsum(hipStream_t s, const float *X, int M, int N, float *out)
{
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, X, M, N, (int64_t)N, out);
    return hipGetLastError();
}

// Forward pass of rows X[0..B) into H1, H2, Y.
hipError_t forward(asp_mlp *n, const float *X, int B, float *Y)
{
    hipStream_t s = n->stream;
    const float *w = n->w;
    hipError_t e;
    if ((e = gemm(s, B, kNetH, kNetIn, X, kNetIn, 1, w, 1, kNetIn, n->H1, kNetH, kEpiBiasRelu,
                  w + kOffB1)) != hipSuccess) return e;
    if ((e = gemm(s, B, kNetH, kNetH, n->H1, kNetH, 1, w + kOffW2, 1, kNetH, n->H2, kNetH,
                  kEpiBiasRelu, w + kOffB2)) != hipSuccess) return e;
    return gemm(s, B, kNetOut, kNetH, n->H2, kNetH, 1, w + kOffW3, 1, kNetH, Y, kNetOut, kEpiBias,
                w + kOffB3);
}

// Loss (added to n->loss) and the full gradient into n->g for the batch in
// n->X, n->T.
hipError_t forward_backward(asp_mlp *n, int B)
{
    hipStream_t s = n->stream;
    const float *w = n->w;
    float *g = n->g;
    hipError_t e;
    if ((e = forward(n, n->X, B, n->Y)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, n->Y, n->T, B * kNetOut, n->dY, n->loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // layer 3: dW3 = dY^T H2, db3 = sum dY, dH2 = (dY W3) * [H2 > 0]
    if ((e = gemm(s, kNetOut, kNetH, B, n->dY, 1, kNetOut, n->H2, kNetH, 1, g + kOffW3, kNetH,
                  kEpiPlain)) != hipSuccess) return e;
    if ((e = colsum(s, n->dY, B, kNetOut, g + kOffB3)) != hipSuccess) return e;
    if ((e = gemm(s, B, kNetH, kNetOut, n->dY, kNetOut, 1, w + kOffW3, kNetH, 1, n->dH2, kNetH,
                  kEpiMask, nullptr, n->H2)) != hipSuccess) return e;
    // layer 2
    if ((e = gemm(s, kNetH, kNetH, B, n->dH2, 1, kNetH, n->H1, kNetH, 1, g + kOffW2, kNetH,
                  kEpiPlain)) != hipSuccess) return e;
    if ((e = colsum(s, n->dH2, B, kNetH, g + kOffB2)) != hipSuccess) return e;
    if ((e = gemm(s, B, kNetH, kNetH, n->dH2, kNetH, 1, w + kOffW2, kNetH, 1, n->dH1, kNetH,
                  kEpiMask, nullptr, n->H1)) != hipSuccess) return e;
    // layer 1
    if ((e = gemm(s, kNetH, kNetIn, B, n->dH1, 1, kNetH, n->X, kNetIn, 1, g, kNetIn,
                  kEpiPlain)) != hipSuccess) return e;
    return colsum(s, n->dH1, B, kNetH, g + kOffB1);
}

hipError_t gather_batch(asp_mlp *n, const float *x, const float *t, int64_t n_rows,
                        const int32_t *idx, int B)
{
    hipStream_t s = n->stream;
    const int64_t nx = (int64_t)B * kNetIn, nt = (int64_t)B * kNetOut;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, x, n_rows,
                       idx, B, kNetIn, n->X, n->bad);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, t, n_rows,
                       idx, B, kNetOut, n->T, n->bad);
    return hipGetLastError();
}

void mlp_release(asp_mlp *n)
{
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    float *bufs[] = {n->w, n->g, n->m, n->v, n->X, n->T, n->H1, n->H2, n->Y, n->dY, n->dH1, n->dH2};
    for (float *b : bufs) (void)hipFree(b);
    (void)hipFree(n->loss);
    (void)hipFree(n->bad);
    if (n->own_stream && n->stream) (void)hipStreamDestroy(n->stream);
}

}  // namespace

extern "C" {

asp_status asp_mlp_create(const float *init, int32_t max_batch, void *stream, asp_mlp **out)
{
    if (!out) return ASP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!init || max_batch < 1 || max_batch > 65536) return ASP_ERR_INVALID_ARG;
    asp_mlp *n = new (std::nothrow) asp_mlp;
    if (!n) return ASP_ERR_NOMEM;
    n->bmax = max_batch;
    auto bail = [&](asp_status s) { mlp_release(n); delete n; return s; };
    if (stream) {
        n->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&n->stream) != hipSuccess) return bail(ASP_ERR_DEVICE);
        n->own_stream = true;
    }
    const size_t P = sizeof(float) * kNetParams;
    const size_t B = (size_t)max_batch;
    if (hipMalloc(&n->w, P) != hipSuccess || hipMalloc(&n->g, P) != hipSuccess ||
        hipMalloc(&n->m, P) != hipSuccess || hipMalloc(&n->v, P) != hipSuccess ||
        hipMalloc(&n->X, sizeof(float) * B * kNetIn) != hipSuccess ||
        hipMalloc(&n->T, sizeof(float) * B * kNetOut) != hipSuccess ||
        hipMalloc(&n->H1, sizeof(float) * B * kNetH) != hipSuccess ||
        hipMalloc(&n->H2, sizeof(float) * B * kNetH) != hipSuccess ||
        hipMalloc(&n->Y, sizeof(float) * B * kNetOut) != hipSuccess ||
        hipMalloc(&n->dY, sizeof(float) * B * kNetOut) != hipSuccess ||
        hipMalloc(&n->dH1, sizeof(float) * B * kNetH) != hipSuccess ||
        hipMalloc(&n->dH2, sizeof(float) * B * kNetH) != hipSuccess ||
        hipMalloc(&n->loss, sizeof(double)) != hipSuccess ||
        hipMalloc(&n->bad, sizeof(int32_t)) != hipSuccess)
        return bail(ASP_ERR_NOMEM);
    if (hipMemcpyAsync(n->w, init, P, hipMemcpyHostToDevice, n->stream) != hipSuccess ||
        hipMemsetAsync(n->m, 0, P, n->stream) != hipSuccess ||
        hipMemsetAsync(n->v, 0, P, n->stream) != hipSuccess ||
        hipStreamSynchronize(n->stream) != hipSuccess)
        return bail(ASP_ERR_DEVICE);
    *out = n;
    return ASP_OK;
}

void asp_mlp_destroy(asp_mlp *n)
{
    mlp_release(n);
    delete n;
}

const char *asp_mlp_last_error(const asp_mlp *n)
{
    return n ? n->err.c_str() : "null network";
}

asp_status asp_mlp_weights(asp_mlp *n, float *out)
{
    if (!n || !out) return ASP_ERR_INVALID_ARG;
    MLP_HIP(n, hipMemcpyAsync(out, n->w, sizeof(float) * kNetParams, hipMemcpyDeviceToHost,
                              n->stream));
    MLP_HIP(n, hipStreamSynchronize(n->stream));
    return ASP_OK;
}

asp_status asp_mlp_loss_grad(asp_mlp *n, const float *x_dev, const float *t_dev, int32_t batch,
                             double *loss, float *grad)
{
    if (!n || !x_dev || !t_dev || batch < 1 || batch > n->bmax) return ASP_ERR_INVALID_ARG;
    const int64_t nx = (int64_t)batch * kNetIn, nt = (int64_t)batch * kNetOut;
    MLP_HIP(n, hipMemcpyAsync(n->X, x_dev, sizeof(float) * nx, hipMemcpyDeviceToDevice, n->stream));
    MLP_HIP(n, hipMemcpyAsync(n->T, t_dev, sizeof(float) * nt, hipMemcpyDeviceToDevice, n->stream));
    MLP_HIP(n, hipMemsetAsync(n->loss, 0, sizeof(double), n->stream));
    MLP_HIP(n, forward_backward(n, batch));
    if (grad)
        MLP_HIP(n, hipMemcpyAsync(grad, n->g, sizeof(float) * kNetParams, hipMemcpyDeviceToHost,
                                  n->stream));
    double l = 0.0;
    MLP_HIP(n, hipMemcpyAsync(&l, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    MLP_HIP(n, hipStreamSynchronize(n->stream));
    if (loss) *loss = l;
    return ASP_OK;
}

asp_status asp_mlp_train(asp_mlp *n, const float *x_dev, const float *t_dev, int64_t n_rows,
                         const int32_t *order_dev, int64_t n_steps, int32_t batch, float lr,
                         double *mean_loss)
{
    if (!n || !x_dev || !t_dev || !order_dev || n_rows < 1 || n_steps < 0 || batch < 1 ||
        batch > n->bmax || !(lr > 0.0f))
        return ASP_ERR_INVALID_ARG;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    MLP_HIP(n, hipMemsetAsync(n->loss, 0, sizeof(double), n->stream));
    MLP_HIP(n, hipMemsetAsync(n->bad, 0, sizeof(int32_t), n->stream));
    for (int64_t st = 0; st < n_steps; ++st) {
        MLP_HIP(n, gather_batch(n, x_dev, t_dev, n_rows, order_dev + st * batch, batch));
        MLP_HIP(n, forward_backward(n, batch));
        n->t += 1;
        const float c1 = (float)(1.0 / (1.0 - pow(0.9, (double)n->t)));
        const float c2 = (float)(1.0 / (1.0 - pow(0.999, (double)n->t)));
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((kNetParams + 255) / 256)), dim3(256), 0,
                           n->stream, n->w, n->m, n->v, n->g, kNetParams, lr, beta1, beta2, eps,
                           c1, c2);
        MLP_HIP(n, hipGetLastError());
    }
    double l = 0.0;
    int32_t bad = 0;
    MLP_HIP(n, hipMemcpyAsync(&l, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    MLP_HIP(n, hipMemcpyAsync(&bad, n->bad, sizeof(int32_t), hipMemcpyDeviceToHost, n->stream));
    MLP_HIP(n, hipStreamSynchronize(n->stream));
    if (mean_loss) *mean_loss = n_steps > 0 ? l / (double)n_steps : 0.0;
    if (bad) return mfail(n, ASP_ERR_INVALID_ARG, "a sample index lies outside the data");
    return ASP_OK;
}

asp_status asp_mlp_forward(asp_mlp *n, const float *x_dev, int64_t rows, float *y_dev)
{
    if (!n || (!x_dev && rows > 0) || (!y_dev && rows > 0) || rows < 0) return ASP_ERR_INVALID_ARG;
    for (int64_t r = 0; r < rows; r += n->bmax) {
        const int B = (int)((rows - r) < n->bmax ? (rows - r) : n->bmax);
        MLP_HIP(n, forward(n, x_dev + r * kNetIn, B, y_dev + r * kNetOut));
    }
    MLP_HIP(n, hipStreamSynchronize(n->stream));
    return ASP_OK;
}

}  // extern "C"
