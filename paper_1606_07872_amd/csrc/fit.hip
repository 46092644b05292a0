// The active-set Levenberg-Marquardt fit of the Asp-Clean2016 minor cycle
// (Zhang, Bhatnagar, Rau & Zhang 2016, Sect. 3, Eq. 4) spread over the whole
// GPU.
//
// One cooperative launch, one work-group per CU.  Work-group 0 owns the fit:
// it takes the peak, applies the stop test (Sect. 2 step 4), forms the start
// values (the simple initial values of Sect. 3, or a clamped proposal),
// selects the active set, keeps the LM state in its LDS, and after every
// trial reduces, solves and publishes the next trial point.  Every LM trial
// evaluates
//     F(theta) = sum_{U(theta)} M (M - 2 D),   H = J^T J,   g = J^T (D - M)
// over U(theta), the union of the members' windows at theta (a truncated
// Gaussian is zero outside its window, so F is the whole-image objective of
// Eq. 4 up to a constant); D is the residual with the old members' stored
// Gaussians added back.  The 256-pixel tiles of U are dealt to the first
// geff work-groups.  Per pixel, D, M, the residual r = D - M and M (M - 2 D)
// are formed in FP64 (r is a small difference of O(1) terms); J and r go to
// FP32 for the augmented Gram matrix [J r]^T [J r], summed per tile and
// Kahan-compensated across tiles, while F and chi2 stay FP64.
//
// Every work-group arrives once per round: at its group's counter (kGroup
// work-groups), the last of a group sums the group's partial rows in order and
// arrives at the top counter; work-group 0 waits for all groups, so no
// work-group can fall a round behind.  Every wait is bounded; a wait that runs
// out marks the context with ASP_ERR_DEVICE and every work-group leaves.
#include <math.h>

#include "asp_device.h"
#include "cycle.h"

namespace asp {

constexpr int kT = kFitThreads;
constexpr int kOwnMax = (kNOutMax + kT - 1) / kT;
constexpr size_t kTileBytes = sizeof(float) * kT * kTileStride;
constexpr size_t kMatBytes = sizeof(double) * kMaxN * kMaxN;
constexpr size_t kFitLds = kTileBytes + 2 * kMatBytes;   // tile (or A) | two Gram buffers
constexpr int kGroup = 16;        // work-groups per first-level arrival group
static_assert(kTileBytes >= kMatBytes, "A shares the tile buffer");
static_assert(kTileBytes >= sizeof(float) * kUpdTabFloats, "the update's tables share the tile buffer");

// Phase timer slots of DevState::prof.
enum { kPCheckin = 0, kPSetup, kPEval, kPWait, kPReduce, kPLmStep, kPCommit, kPPrepare,
       kPArrive, kPTrials, kPFits, kPEvalPx, kPSoloTrials, kPSoloPx };
static_assert(kPSoloPx + 1 == kProfSlots, "profile slots");

__device__ inline unsigned long long now_ticks() { return wall_clock64(); }

// Polling loops sleep this many units of 64 clocks between reads of a
// counter another work-group advances (fewer reads of one line while waiting).
constexpr int kPollSleep = 8;

struct WGShared {
    // member constants at the parameters under evaluation
    int32_t win[kMaxM][4], wold[kMaxM][4];
    int64_t pref[kMaxM + 1];
    double mx[kMaxM], my[kMaxM], mamp[kMaxM], minv2[kMaxM], minvs2[kMaxM], minvs3[kMaxM];
    double ox[kMaxM], oy[kMaxM], oamp[kMaxM], oinv2[kMaxM];
    int32_t m, n;
    double wsum[4][3];
    double wred[kT / 64][48];
    // the reduced trial (work-group 0)
    double ge[kMaxN], Fe, chi2e;
    int64_t npx_e;
    // LM state (work-group 0)
    double th_c[kMaxN], th_e[kMaxN], g_c[kMaxN], lo[kMaxN], hi[kMaxN], th0[kMaxN], th_old[kMaxN];
    double dd[kMaxN], rhs[kMaxN], rhs_copy[kMaxN], delta[kMaxN];
    double ldiag[kMaxN];           // L_kk of the work-group Cholesky
    int32_t frozen[kMaxN];
    double F_c, chi2_c, mu, nu, pred, chi2_init, peak;
    int32_t trials, trials_total, converged, used_fallback, use_prop, pass, phase;
    int32_t members[kMaxM];
    int64_t idx, npx_c;
    // selection scratch
    uint32_t mask[kT];
    double t0[4];                  // the start of the new component (simple or smoothing)
    double alt[4];                 // a proposal start, compared with t0 by the objective
    int32_t alt_pending, chose_prop;
    int32_t hsel;                  // which of the two Gram buffers holds the current point
    double sel[3];                 // (x, y, s) of the start: the active set is selected around it
    int32_t use_smooth;            // the start is the smoothing method's
    int32_t nch, sel_done;
    unsigned long long key;        // the peak key of this fit (collect_peak_key)
    // batched fields (leader and followers)
    int32_t cmd, fld, go;
    int64_t k_target, upx;
    // control
    unsigned long long tmark;      // phase timer mark (thread 0)
    unsigned long long tfit;       // start of the fit (thread 0)
    unsigned int gen;
    int32_t last, abort, done, ok, finished, accept, stop;
    int32_t upd;                   // the fit committed and this launch also updates R
};

// Phase timers of the driving work-group (thread 0): the mark lives in LDS so
// that no tick value stays in registers across a phase.
__device__ inline void mark(WGShared &S)
{
    if (threadIdx.x == 0) S.tmark = now_ticks();
}

__device__ __forceinline__ void lap(const Params &p, WGShared &S, int slot)
{
    if (threadIdx.x == 0) {
        const unsigned long long now = now_ticks();
        atomicAdd(&p.st->prof[slot], now - S.tmark);
        S.tmark = now;
    }
}

// ---------------------------------------------------------------------------
// Synchronisation between work-groups.  Polling is relaxed (no cache
// maintenance per poll); the fence after it is the acquire.  A work-group
// signals after a barrier, by one release operation of thread 0.
// ---------------------------------------------------------------------------

__device__ inline void acquire_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Loads of data another work-group published: agent-scope atomic loads read
// the coherent copy, so a reader that only needs such data can skip the
// acquire fence (which would also drop the read-only residual from its L2).
__device__ inline double ld_shared(const double *q)
{
    return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int32_t ld_shared(const int32_t *q)
{
    return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wait is bounded in time: `limit` device wall-clock ticks.  With
// `beat`, the bound restarts whenever the heartbeat moves: a leader that
// works alone for a long time (small fields of a batch) keeps its followers
// waiting without letting them time out.
__device__ __forceinline__ bool wait_publish(FitGlobal *G, WGShared &S, unsigned long long limit,
                                             bool acquire = true, bool beat = false)
{
    if (threadIdx.x == 0) {
        unsigned int now = S.gen;
        unsigned int last_beat = beat ? __hip_atomic_load(&G->beat, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) : 0u;
        unsigned long long t0 = now_ticks();
        for (;;) {
            now = __hip_atomic_load(&G->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (now != S.gen) break;
            const unsigned long long tn = now_ticks();
            if (beat) {
                const unsigned int b = __hip_atomic_load(&G->beat, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                if (b != last_beat) { last_beat = b; t0 = tn; }
            }
            if (tn - t0 > limit) break;
            __builtin_amdgcn_s_sleep(kPollSleep);
        }
        S.abort = (now == S.gen) ? 1 : 0;
        S.gen = now;
        if (acquire) acquire_fence();
    }
    __syncthreads();
    return S.abort == 0;
}

// The barrier makes every thread's stores visible to thread 0, whose release
// at agent scope then covers them (the pattern of a grid-wide barrier).
__device__ __forceinline__ void publish(FitGlobal *G)
{
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&G->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *ctr reaches target; returns false on timeout.
__device__ __forceinline__ bool spin_until(unsigned int *ctr, unsigned int target,
                                           unsigned long long limit, bool acquire = true)
{
    const unsigned long long t0 = now_ticks();
    bool ok = true;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (now_ticks() - t0 > limit) { ok = false; break; }
        __builtin_amdgcn_s_sleep(kPollSleep);
    }
    if (acquire) acquire_fence();
    return ok;
}

// ---------------------------------------------------------------------------
// Active set (the paper names the heuristic; its definition is in the 2004
// paper).  Candidates are components whose amplitude has the peak's sign and
// whose centre lies inside the window of the simple start (the peak pixel,
// width omega_b), most recent first; skip one closer than
// max(omega_b, min(s_j, s_m)) to a member already taken (the new component
// first: at the peak pixel with width omega_b and, with a proposal, at the
// proposal too); at most K_max - 1.  FP64 products and sums are rounded
// separately, so membership is reproducible bit for bit.
// ---------------------------------------------------------------------------

__device__ inline bool too_close(double xj, double yj, double sj, double xm, double ym,
                                 double sm, double omega_b)
{
    double ex = __dsub_rn(xj, xm), ey = __dsub_rn(yj, ym);
    double rs = sj < sm ? sj : sm;
    if (rs < omega_b) rs = omega_b;
    return __dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)) <= __dmul_rn(rs, rs);
}

// Lane 0 of wave 0: greedy acceptance of candidate j.
__device__ __forceinline__ void consider(const Params &p, WGShared &S, int64_t j, double omega_b)
{
    const double xj = p.cx[j], yj = p.cy[j], sj = p.cs[j];
    if (too_close(xj, yj, sj, S.sel[0], S.sel[1], S.sel[2], omega_b)) return;
    // a proposal start is a second place of the new component
    if (S.alt_pending && too_close(xj, yj, sj, S.alt[1], S.alt[2], S.alt[3], omega_b)) return;
    for (int u = 0; u < S.nch; ++u) {
        const int64_t mj = S.members[u + 1];
        if (too_close(xj, yj, sj, p.cx[mj], p.cy[mj], p.cs[mj], omega_b)) return;
    }
    S.members[1 + S.nch] = (int32_t)j;
    S.nch++;
    if (S.nch >= p.max_active - 1) S.sel_done = 1;
}

// Start values, active set, bounds; the start point goes to S.th_e and is
// published in G.  Work-group 0, whole work-group.
__device__ __forceinline__ void setup_fit(const Params &p, FitGlobal *G, WGShared &S, bool use_prop)
{
    const int t = threadIdx.x;
    const double omega_b = p.st->omega_b;
    if (t == 0) {
        const int64_t pr = S.idx / p.W, pc = S.idx % p.W;
        const double pv = S.peak;
        double *t0 = S.t0;
        const double cap = width_cap(p);
        if (S.use_smooth) {
            // the smoothing method's start (Sect. 2 step 1, Sect. 3)
            const double *q = p.st->smooth_start;
            t0[0] = q[0]; t0[1] = q[1]; t0[2] = q[2]; t0[3] = q[3];
        } else {
            t0[0] = pv; t0[1] = (double)pc; t0[2] = (double)pr; t0[3] = omega_b;
        }
        S.alt_pending = use_prop ? 1 : 0;
        S.chose_prop = 0;
        if (use_prop) {
            // the proposal, clamped: the peak's sign, within 16 px of the peak
            // and inside the image, omega_b <= s <= the width cap
            const double *q = p.st->proposal;
            double *a = S.alt;
            a[0] = q[0]; a[1] = q[1]; a[2] = q[2]; a[3] = q[3];
            if (!(a[0] * pv > 0.0)) a[0] = pv;     // also NaN
            if (!(a[1] >= (double)pc - 16.0)) a[1] = (double)pc - 16.0;
            if (a[1] > (double)pc + 16.0) a[1] = (double)pc + 16.0;
            if (!(a[2] >= (double)pr - 16.0)) a[2] = (double)pr - 16.0;
            if (a[2] > (double)pr + 16.0) a[2] = (double)pr + 16.0;
            if (a[1] < 0.0) a[1] = 0.0;
            if (a[1] > (double)(p.W - 1)) a[1] = (double)(p.W - 1);
            if (a[2] < 0.0) a[2] = 0.0;
            if (a[2] > (double)(p.H - 1)) a[2] = (double)(p.H - 1);
            if (!(a[3] >= omega_b)) a[3] = omega_b;
            if (a[3] > cap) a[3] = cap;
        }
        // candidates: inside the start's window (the simple start, peak pixel
        // and omega_b, also when a proposal competes; or the smoothing start)
        S.sel[0] = t0[1];
        S.sel[1] = t0[2];
        S.sel[2] = t0[3];
        make_window(t0[1], t0[2], halfwidth(t0[3], p.window_sigmas), p.H, p.W, S.win[0]);
        S.nch = 0;
        S.sel_done = (p.max_active <= 1) ? 1 : 0;
    }
    __syncthreads();
    const double a0 = S.t0[0];
    const int32_t b0 = S.win[0][0], b1 = S.win[0][1], b2 = S.win[0][2], b3 = S.win[0][3];
    const int64_t L = p.st->L;
    constexpr int64_t kSeg = (int64_t)kT * 32;
    for (int64_t top = L; top > 0; top -= kSeg) {
        __syncthreads();
        if (S.sel_done) break;
        const int64_t lo = top - kSeg > 0 ? top - kSeg : 0;
        S.mask[t] = 0u;
        __syncthreads();
        for (int64_t j = lo + t; j < top; j += kT) {
            const double aj = p.ca[j];
            if (!(__dmul_rn(aj, a0) > 0.0)) continue;
            const double xj = p.cx[j], yj = p.cy[j];
            if (!(yj >= (double)b0 && yj <= (double)b1 && xj >= (double)b2 && xj <= (double)b3))
                continue;
            const int64_t o = j - lo;
            atomicOr(&S.mask[o >> 5], 1u << (o & 31));
        }
        __syncthreads();
        if (t < 64) {
            // words from the highest index down: lane l holds word wbase + 63 - l
            for (int wbase = kT - 64; wbase >= 0; wbase -= 64) {
                const uint32_t word = S.mask[wbase + 63 - t];
                unsigned long long nz = __ballot(word != 0u);
                while (nz) {
                    const int l = __ffsll((long long)nz) - 1;
                    nz &= nz - 1ull;
                    const uint32_t wv = __shfl(word, l, 64);
                    if (t == 0 && !S.sel_done) {
                        uint32_t bits = wv;
                        while (bits && !S.sel_done) {
                            const int b = 31 - __clz(bits);
                            bits &= ~(1u << b);
                            consider(p, S, lo + 32 * (wbase + 63 - l) + b, omega_b);
                        }
                    }
                    if (__shfl(S.sel_done, 0, 64)) break;
                }
                if (__shfl(S.sel_done, 0, 64)) break;
            }
        }
    }
    __syncthreads();
    const int m = 1 + S.nch;
    if (t == 0) {
        S.members[0] = -1;
        S.hsel = 0;
        S.m = m;
        S.n = 4 * m;
        S.phase = 0;
        S.trials = 0;
        S.converged = 0;
        G->m = m;
        G->n = 4 * m;
    }
    __syncthreads();
    if (t < m) {
        double th[4];
        if (t == 0) {
            th[0] = S.t0[0]; th[1] = S.t0[1]; th[2] = S.t0[2]; th[3] = S.t0[3];
        } else {
            const int64_t j = S.members[t];
            th[0] = p.ca[j]; th[1] = p.cx[j]; th[2] = p.cy[j]; th[3] = p.cs[j];
        }
        int32_t w[4];
        make_window(th[1], th[2], halfwidth(th[3], p.window_sigmas), p.H, p.W, w);
        if (t == 0 && S.alt_pending) {
            // two starts: the centre may range over the hull of both windows
            int32_t wa[4];
            make_window(S.alt[1], S.alt[2], halfwidth(S.alt[3], p.window_sigmas), p.H, p.W, wa);
            w[0] = wa[0] < w[0] ? wa[0] : w[0];
            w[1] = wa[1] > w[1] ? wa[1] : w[1];
            w[2] = wa[2] < w[2] ? wa[2] : w[2];
            w[3] = wa[3] > w[3] ? wa[3] : w[3];
        }
        // bounds: the start sign of the amplitude; the centre inside its start
        // window; omega_b <= s <= the width cap
        const bool neg = th[0] < 0.0;
        const double lo4[4] = {neg ? -INFINITY : 0.0, (double)w[2], (double)w[0], omega_b};
        const double hi4[4] = {neg ? 0.0 : INFINITY, (double)w[3], (double)w[1], width_cap(p)};
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * t + q;
            S.lo[i] = lo4[q];
            S.hi[i] = hi4[q];
            S.th0[i] = th[q];
            S.th_old[i] = (t == 0) ? 0.0 : th[q];
            double v = th[q];
            if (!(v >= lo4[q])) v = lo4[q];
            if (v > hi4[q]) v = hi4[q];
            S.th_e[i] = v;
            G->th_e[i] = v;
            G->th_old[i] = S.th_old[i];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Evaluation of one work-group's share of U(theta).
// ---------------------------------------------------------------------------

// Entry o of the augmented Gram matrix [J r]^T [J r]: the upper triangle of
// the columns 0..n (J then the residual), row by row.
__device__ inline void out_pair(int o, int n, int &i, int &k)
{
    int r = 0, start = 0;
    while (start + (n + 1 - r) <= o) { start += n + 1 - r; ++r; }
    i = r;
    k = r + (o - start);
}

// Member constants at theta (th_e) and the old members' stored Gaussians
// (th_old), from the published copy or from work-group 0's own.
__device__ __forceinline__ void prepare(const Params &p, WGShared &S, int m, const double *th_e,
                                        const double *th_old, bool published = false)
{
    const int t = threadIdx.x;
    __syncthreads();
    if (t == 0) { S.m = m; S.n = 4 * m; }
    __syncthreads();
    if (t < S.m) {
        // published: another work-group's copy in global memory
        auto ld = [&](const double *q) { return published ? ld_shared(q) : *q; };
        const double a = ld(th_e + 4 * t), x = ld(th_e + 4 * t + 1), y = ld(th_e + 4 * t + 2),
                     s = ld(th_e + 4 * t + 3);
        make_window(x, y, halfwidth(s, p.window_sigmas), p.H, p.W, S.win[t]);
        const double s2 = s * s;
        S.mx[t] = x;
        S.my[t] = y;
        S.mamp[t] = a;
        S.minv2[t] = 1.0 / (2.0 * s2);
        S.minvs2[t] = 1.0 / s2;
        S.minvs3[t] = 1.0 / (s2 * s);
        if (t > 0) {
            const double oa = ld(th_old + 4 * t), ox = ld(th_old + 4 * t + 1),
                         oy = ld(th_old + 4 * t + 2), os = ld(th_old + 4 * t + 3);
            make_window(ox, oy, halfwidth(os, p.window_sigmas), p.H, p.W, S.wold[t]);
            S.ox[t] = ox;
            S.oy[t] = oy;
            S.oamp[t] = oa;
            S.oinv2[t] = 1.0 / (2.0 * os * os);
        }
    }
    __syncthreads();
    if (t == 0) {
        S.pref[0] = 0;
        for (int j = 0; j < S.m; ++j)
            S.pref[j + 1] = S.pref[j] + (int64_t)(S.win[j][1] - S.win[j][0] + 1) *
                                            (S.win[j][3] - S.win[j][2] + 1);
    }
    __syncthreads();
}

// Orders the LDS accesses of one wave: the lanes of a wave issue LDS
// instructions together and the LDS serves them in program order, so after
// this point every lane sees what any lane of the wave wrote before it; the
// wavefront-scope fences keep the compiler from moving accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Tiles tile0, tile0 + stride, ... of U; the work-group's partial (FP64:
// n_out Gram entries, F, chi2, the pixel count) goes to out.
__device__ __forceinline__ void evaluate_tiles(const Params &p, WGShared &S, float *tile, double *red,
                               int64_t tile0, int64_t stride, double *out)
{
    const int t = threadIdx.x;
    const int m = S.m, n = S.n;
    const int n_out = (n + 1) * (n + 2) / 2;
    int S_sub = 1, my_s = 0, n_own = 0;
    int oi[kOwnMax], ok_[kOwnMax];
    if (n_out <= kT) {
        S_sub = kT / n_out;
        my_s = t / n_out;
        n_own = my_s < S_sub ? 1 : 0;
        if (n_own) out_pair(t % n_out, n, oi[0], ok_[0]);
    } else {
#pragma unroll
        for (int u = 0; u < kOwnMax; ++u) {
            const int o = t + u * kT;
            if (o < n_out) { out_pair(o, n, oi[u], ok_[u]); n_own = u + 1; }
        }
    }
    float acc_s[kOwnMax], acc_c[kOwnMax];
#pragma unroll
    for (int u = 0; u < kOwnMax; ++u) { acc_s[u] = 0.0f; acc_c[u] = 0.0f; }

    const int64_t total = S.pref[m];
    const int64_t ntiles = (total + kT - 1) / kT;
    double npx = 0.0, f_acc = 0.0, c_acc = 0.0;
    float *row = tile + t * kTileStride;
    // This thread's pixel of tile ti: coordinates, whether it is a first
    // occurrence in U, and its residual value (loaded one tile ahead).
    auto locate = [&](int64_t ti, int32_t &r, int32_t &c, bool &valid, float &rv) {
        const int64_t lin = ti * kT + t;
        valid = false;
        r = 0;
        c = 0;
        rv = 0.0f;
        if (ti >= ntiles || lin >= total) return;
        int w = 0;
        while (lin >= S.pref[w + 1]) ++w;
        // a window lies inside the image (fewer than 2^32 pixels): 32-bit division
        const uint32_t local = (uint32_t)(lin - S.pref[w]);
        const uint32_t wc = (uint32_t)(S.win[w][3] - S.win[w][2] + 1);
        r = S.win[w][0] + (int32_t)(local / wc);
        c = S.win[w][2] + (int32_t)(local % wc);
        valid = true;
        for (int i = 0; i < w; ++i)
            if (in_box(S.win[i], r, c)) { valid = false; break; }
        if (valid) rv = p.R[(int64_t)r * p.W + c];
    };
    int32_t nr_, nc_;
    bool nvalid;
    float nrv;
    locate(tile0, nr_, nc_, nvalid, nrv);
    for (int64_t ti = tile0; ti < ntiles; ti += stride) {
        const int32_t r = nr_, c = nc_;
        const bool valid = nvalid;
        const float rv = nrv;
        locate(ti + stride, nr_, nc_, nvalid, nrv);
        if (valid) {
            npx += 1.0;
            double D = (double)rv;
            const double cd = (double)c, rd = (double)r;
            for (int j = 1; j < m; ++j) {
                if (!in_box(S.wold[j], r, c)) continue;
                const double dx = cd - S.ox[j], dy = rd - S.oy[j];
                D += S.oamp[j] * exp(-(dx * dx + dy * dy) * S.oinv2[j]);
            }
            double M = 0.0;
            for (int j = 0; j < m; ++j) {
                float *J = row + 4 * j;
                if (!in_box(S.win[j], r, c)) { J[0] = J[1] = J[2] = J[3] = 0.0f; continue; }
                const double dx = cd - S.mx[j], dy = rd - S.my[j];
                const double q = dx * dx + dy * dy;
                const double e = exp(-q * S.minv2[j]);
                const double G = S.mamp[j] * e;
                M += G;
                J[0] = (float)e;
                J[1] = (float)(G * dx * S.minvs2[j]);
                J[2] = (float)(G * dy * S.minvs2[j]);
                J[3] = (float)(G * q * S.minvs3[j]);
            }
            const double res = D - M;
            row[n] = (float)res;
            f_acc += M * (M - 2.0 * D);
            c_acc += res * res;
        } else {
            for (int k = 0; k <= n; ++k) row[k] = 0.0f;
        }
        __syncthreads();
        // plain FP32 sum over the tile's pixels, Kahan-compensated across tiles
#pragma unroll
        for (int u = 0; u < kOwnMax; ++u) {
            if (u >= n_own) break;
            const int ci = oi[u], ck = ok_[u];
            // four interleaved chains (pixels q, q + S_sub, ... in turn), added
            // in a fixed order: a quarter of the dependent adds per tile
            float ts0 = 0.0f, ts1 = 0.0f, ts2 = 0.0f, ts3 = 0.0f;
            int q = my_s;
            for (; q + 3 * S_sub < kT; q += 4 * S_sub) {
                const float *r0 = tile + q * kTileStride, *r1 = r0 + S_sub * kTileStride;
                const float *r2 = r1 + S_sub * kTileStride, *r3 = r2 + S_sub * kTileStride;
                ts0 += r0[ci] * r0[ck];
                ts1 += r1[ci] * r1[ck];
                ts2 += r2[ci] * r2[ck];
                ts3 += r3[ci] * r3[ck];
            }
            for (; q < kT; q += S_sub) {
                const float *rq = tile + q * kTileStride;
                ts0 += rq[ci] * rq[ck];
            }
            const float ts = (ts0 + ts1) + (ts2 + ts3);
            const float y = ts - acc_c[u];
            const float tt = acc_s[u] + y;
            acc_c[u] = (tt - acc_s[u]) - y;
            acc_s[u] = tt;
        }
        __syncthreads();
    }
    // the work-group's partial, summed over the pixel subsets in a fixed order
    if (n_out <= kT) {
        red[t] = n_own ? (double)acc_s[0] - (double)acc_c[0] : 0.0;
        __syncthreads();
        if (t < n_out) {
            double v = 0.0;
            for (int s = 0; s < S_sub; ++s) v += red[t + s * n_out];
            out[t] = v;
        }
    } else {
#pragma unroll
        for (int u = 0; u < kOwnMax; ++u) {
            if (u >= n_own) break;
            out[t + u * kT] = (double)acc_s[u] - (double)acc_c[u];
        }
    }
    // F, chi2 and the pixel count: wave sums, then the four waves in order
    const double f_w = wave_sum(f_acc), c_w = wave_sum(c_acc), p_w = wave_sum(npx);
    if ((t & 63) == 0) {
        S.wsum[t >> 6][0] = f_w;
        S.wsum[t >> 6][1] = c_w;
        S.wsum[t >> 6][2] = p_w;
    }
    __syncthreads();
    if (t < 3) {
        double v = 0.0;
        for (int w = 0; w < kT / 64; ++w) v += S.wsum[w][t];
        out[n_out + t] = v;
    }
    __syncthreads();
}

// The same partial for fits of three or more members with the Gram sums on
// the matrix cores.  The tile of [J r] rows is formed in LDS exactly as above.
// Wave w then takes pixel rows 64w .. 64w+63 of the tile and accumulates
// G = X^T X over them with v_mfma_f32_16x16x4f32 (four pixels per
// instruction), one 16 x 16 block per pair of 16-column groups (bi >= bj) of
// X; columns past n are read as zeros.  A tile's FP32 block sums are added
// into FP64 accumulators, so the sums across tiles lose nothing.  At the end
// the four waves' FP64 sums are added through LDS in a fixed order:
// (w0 + w2) + (w1 + w3).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NB>
__device__ void evaluate_tiles_mfma(const Params &p, WGShared &S, float *tile, int64_t tile0,
                                    int64_t stride, double *out)
{
    constexpr int NBL = NB * (NB + 1) / 2;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m = S.m, n = S.n, C = n + 1;
    const int n_out = C * (C + 1) / 2;
    double g[NBL][4];
#pragma unroll
    for (int q = 0; q < NBL; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[q][r] = 0.0;

    const int64_t total = S.pref[m];
    const int64_t ntiles = (total + kT - 1) / kT;
    double npx = 0.0, f_acc = 0.0, c_acc = 0.0;
    float *row = tile + t * kTileStride;
    // This thread's pixel of tile ti: coordinates, whether it is a first
    // occurrence in U, and its residual value (loaded one tile ahead).
    auto locate = [&](int64_t ti, int32_t &r, int32_t &c, bool &valid, float &rv) {
        const int64_t lin = ti * kT + t;
        valid = false;
        r = 0;
        c = 0;
        rv = 0.0f;
        if (ti >= ntiles || lin >= total) return;
        int w = 0;
        while (lin >= S.pref[w + 1]) ++w;
        // a window lies inside the image (fewer than 2^32 pixels): 32-bit division
        const uint32_t local = (uint32_t)(lin - S.pref[w]);
        const uint32_t wc = (uint32_t)(S.win[w][3] - S.win[w][2] + 1);
        r = S.win[w][0] + (int32_t)(local / wc);
        c = S.win[w][2] + (int32_t)(local % wc);
        valid = true;
        for (int i = 0; i < w; ++i)
            if (in_box(S.win[i], r, c)) { valid = false; break; }
        if (valid) rv = p.R[(int64_t)r * p.W + c];
    };
    int32_t nr_, nc_;
    bool nvalid;
    float nrv;
    locate(tile0, nr_, nc_, nvalid, nrv);
    const int kr = lane >> 4, cc = lane & 15;
    for (int64_t ti = tile0; ti < ntiles; ti += stride) {
        const int32_t r = nr_, c = nc_;
        const bool valid = nvalid;
        const float rv = nrv;
        locate(ti + stride, nr_, nc_, nvalid, nrv);
        if (valid) {
            npx += 1.0;
            double D = (double)rv;
            const double cd = (double)c, rd = (double)r;
            for (int j = 1; j < m; ++j) {
                if (!in_box(S.wold[j], r, c)) continue;
                const double dx = cd - S.ox[j], dy = rd - S.oy[j];
                D += S.oamp[j] * exp(-(dx * dx + dy * dy) * S.oinv2[j]);
            }
            double M = 0.0;
            for (int j = 0; j < m; ++j) {
                float *J = row + 4 * j;
                if (!in_box(S.win[j], r, c)) { J[0] = J[1] = J[2] = J[3] = 0.0f; continue; }
                const double dx = cd - S.mx[j], dy = rd - S.my[j];
                const double q = dx * dx + dy * dy;
                const double e = exp(-q * S.minv2[j]);
                const double G = S.mamp[j] * e;
                M += G;
                J[0] = (float)e;
                J[1] = (float)(G * dx * S.minvs2[j]);
                J[2] = (float)(G * dy * S.minvs2[j]);
                J[3] = (float)(G * q * S.minvs3[j]);
            }
            const double res = D - M;
            row[n] = (float)res;
            f_acc += M * (M - 2.0 * D);
            c_acc += res * res;
        } else {
            for (int k = 0; k <= n; ++k) row[k] = 0.0f;
        }
        __syncthreads();
        f32x4 acc[NBL];
#pragma unroll
        for (int q = 0; q < NBL; ++q) acc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
            const float *xr = tile + (wave * 64 + ks * 4 + kr) * kTileStride;
            float x[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int col = b * 16 + cc;
                x[b] = col < C ? xr[col] : 0.0f;
            }
            int q = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj, ++q)
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[bi], x[bj], acc[q], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < NBL; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) g[q][r] += (double)acc[q][r];
        __syncthreads();                   // the tile is rewritten next
    }
    // Lane l of wave w holds, for block (bi, bj), the entries of rows
    // 16 bi + 4 (l / 16) + r and column 16 bj + l % 16 of G.  Entry (i, k),
    // i <= k, of the output is G[k][i], taken from block (k / 16, i / 16).
    double *buf = reinterpret_cast<double *>(tile);
    static_assert(2 * sizeof(double) * (kMaxN + 1) * (kMaxN + 2) / 2 <= kTileBytes, "wave sums");
    for (int half = 0; half < 2; ++half) {
        if ((wave >> 1) == half) {
            double *dst = buf + (wave & 1) * n_out;
            int q = 0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj, ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = 16 * bi + 4 * kr + r, i = 16 * bj + cc;
                        if (k < C && i <= k) {
                            const int o = i * C - i * (i - 1) / 2 + (k - i);
                            dst[o] = half ? dst[o] + g[q][r] : g[q][r];
                        }
                    }
        }
        __syncthreads();
    }
    for (int o = t; o < n_out; o += kT) out[o] = buf[o] + buf[n_out + o];
    // F, chi2 and the pixel count: wave sums, then the four waves in order
    const double f_w = wave_sum(f_acc), c_w = wave_sum(c_acc), p_w = wave_sum(npx);
    if (lane == 0) {
        S.wsum[wave][0] = f_w;
        S.wsum[wave][1] = c_w;
        S.wsum[wave][2] = p_w;
    }
    __syncthreads();
    if (t < 3) {
        double v = 0.0;
        for (int w = 0; w < kT / 64; ++w) v += S.wsum[w][t];
        out[n_out + t] = v;
    }
    __syncthreads();
}

// The same partial for fits of at most two members (n <= 8): each thread keeps
// the 15 or 45 Gram entries of its own pixels in registers, with no barrier per
// tile.  J and r are FP32 values; their products are exact in FP64 and are
// accumulated there (one FP64 FMA per entry, half the work of a Kahan update
// in FP32 on this hardware and a smaller error).  The threads' sums are
// combined once at the end by wave shuffles and the four waves in order.
template <int M>
__device__ __forceinline__ void evaluate_tiles_reg(const Params &p, WGShared &S, int64_t tile0, int64_t stride,
                                   double *out, float *stage)
{
    constexpr int N = 4 * M, C = N + 1, NO = C * (C + 1) / 2;
    const int t = threadIdx.x;
    const int64_t total = S.pref[M];
    const int64_t ntiles = (total + kT - 1) / kT;
    // This thread's pixel of tile ti (row-major within the window it falls in).
    auto locate = [&](int64_t lin, int &w, int32_t &r, int32_t &c) {
        w = (M > 1 && lin >= S.pref[1]) ? 1 : 0;
        // a window lies inside the image (fewer than 2^32 pixels): 32-bit division
        const uint32_t local = (uint32_t)(lin - S.pref[w]);
        const uint32_t wc = (uint32_t)(S.win[w][3] - S.win[w][2] + 1);
        r = S.win[w][0] + (int32_t)(local / wc);
        c = S.win[w][2] + (int32_t)(local % wc);
    };
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    double npx = 0.0, f_acc = 0.0, c_acc = 0.0;
    for (int64_t ti = tile0; ti < ntiles; ti += stride) {
        const int64_t lin = ti * kT + t;
        if (lin >= total) continue;
        int w;
        int32_t r, c;
        locate(lin, w, r, c);
        if (M > 1 && w == 1 && in_box(S.win[0], r, c)) continue;
        npx += 1.0;
        double D = (double)p.R[(int64_t)r * p.W + c];
        const double cd = (double)c, rd = (double)r;
        if (M > 1 && in_box(S.wold[1], r, c)) {
            const double dx = cd - S.ox[1], dy = rd - S.oy[1];
            D += S.oamp[1] * exp(-(dx * dx + dy * dy) * S.oinv2[1]);
        }
        float col[C];
        double Mv = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (!in_box(S.win[j], r, c)) {
                col[4 * j] = col[4 * j + 1] = col[4 * j + 2] = col[4 * j + 3] = 0.0f;
                continue;
            }
            const double dx = cd - S.mx[j], dy = rd - S.my[j];
            const double q = dx * dx + dy * dy;
            const double e = exp(-q * S.minv2[j]);
            const double G = S.mamp[j] * e;
            Mv += G;
            col[4 * j] = (float)e;
            col[4 * j + 1] = (float)(G * dx * S.minvs2[j]);
            col[4 * j + 2] = (float)(G * dy * S.minvs2[j]);
            col[4 * j + 3] = (float)(G * q * S.minvs3[j]);
        }
        const double res = D - Mv;
        col[N] = (float)res;
        f_acc += Mv * (Mv - 2.0 * D);
        c_acc += res * res;
        double cold[C];
#pragma unroll
        for (int i = 0; i < C; ++i) cold[i] = (double)col[i];
        int o = 0;
#pragma unroll
        for (int i = 0; i < C; ++i)
#pragma unroll
            for (int k = i; k < C; ++k, ++o) acc[o] = fma(cold[i], cold[k], acc[o]);
    }
    const int lane = t & 63, wave = t >> 6;
    // Wave sums of the Gram entries, F, chi2 and the pixel count, through the
    // tile buffer (idle in this path): each wave writes its lanes' values,
    // half of them at a time, and lane q then adds value q over the 64 lanes
    // in lane order.  Rows are padded to 65 doubles against bank conflicts.
    constexpr int NV = NO + 3, HALF = (NV + 1) / 2, ROW = 65;
    static_assert(sizeof(double) * (kT / 64) * HALF * ROW <= kTileBytes, "reduction buffer");
    double v[NV];
#pragma unroll
    for (int o = 0; o < NO; ++o) v[o] = acc[o];
    v[NO] = f_acc;
    v[NO + 1] = c_acc;
    v[NO + 2] = npx;
    double *buf = reinterpret_cast<double *>(stage) + wave * (HALF * ROW);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < HALF; ++q)
            if (h * HALF + q < NV) buf[q * ROW + lane] = v[h * HALF + q];
        wave_lds_sync();
        if (lane < HALF && h * HALF + lane < NV) {
            // four interleaved chains over the lanes, added in a fixed order
            const double *row = buf + lane * ROW;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            for (int l = 0; l < 16; ++l) {
                s0 += row[l];
                s1 += row[l + 16];
                s2 += row[l + 32];
                s3 += row[l + 48];
            }
            S.wred[wave][h * HALF + lane] = (s0 + s1) + (s2 + s3);
        }
        wave_lds_sync();                   // the buffer is rewritten by the next half
    }
    __syncthreads();
    if (t < NO + 3) {
        double tot = 0.0;
        for (int wv = 0; wv < kT / 64; ++wv) tot += S.wred[wv][t];
        out[t] = tot;
    }
    __syncthreads();
}

// Rows w0..w1-1 of the partials summed in row order.
__device__ __forceinline__ double sum_column(const Params &p, int w0, int w1, int o)
{
    double v = 0.0;
    int w = w0;
    for (; w + 4 <= w1; w += 4) {
        const double a = ld_shared(p.partials + (int64_t)w * kPartStride + o);
        const double b = ld_shared(p.partials + (int64_t)(w + 1) * kPartStride + o);
        const double c = ld_shared(p.partials + (int64_t)(w + 2) * kPartStride + o);
        const double d = ld_shared(p.partials + (int64_t)(w + 3) * kPartStride + o);
        v += a; v += b; v += c; v += d;
    }
    for (; w < w1; ++w) v += ld_shared(p.partials + (int64_t)w * kPartStride + o);
    return v;
}

__device__ __forceinline__ void sum_rows(const Params &p, int n, int w0, int w1, int dst)
{
    const int n_out = (n + 1) * (n + 2) / 2;
    for (int o = threadIdx.x; o < n_out + 3; o += kT)
        p.partials[(int64_t)dst * kPartStride + o] = sum_column(p, w0, w1, o);
}

// Rows w0..w1-1 summed in row order into He, S.ge, S.Fe, S.chi2e, S.npx_e.
__device__ __forceinline__ void reduce_partials(const Params &p, WGShared &S, int w0, int w1, double *He)
{
    const int n = S.n;
    const int n_out = (n + 1) * (n + 2) / 2;
    for (int o = threadIdx.x; o < n_out + 3; o += kT) {
        const double v = sum_column(p, w0, w1, o);
        if (o >= n_out) {
            if (o == n_out) S.Fe = v;
            else if (o == n_out + 1) S.chi2e = v;
            else S.npx_e = (int64_t)v;
            continue;
        }
        int i, k;
        out_pair(o, n, i, k);
        if (i < n && k < n) { He[i * n + k] = v; He[k * n + i] = v; }
        else if (i < n) S.ge[i] = v;
    }
    __syncthreads();
}

// Work-group Cholesky solve of A x = b (A n x n in LDS, overwritten; b
// overwritten), n <= 64, in the textbook arithmetic: L_kk = sqrt(d_k),
// L_ik = A_ik / L_kk, A_ij -= L_ik L_jk, then the two triangular solves with
// divisions by L_kk.  Column k of L is written into row k of the upper
// triangle (U[k][i] = L[i][k]); the diagonal keeps the pivots d_k and the
// L_kk go to S.ldiag.  Every thread takes the square root itself, so a column
// costs two barriers (after the scaled column, after the trailing update,
// which the threads share as a 16 x 16 grid).  The triangular solves run on
// wave 0, one lane per row, with no barrier.
__device__ bool chol_solve(WGShared &S, double *A, int n, double *b, double *x)
{
    static_assert(kMaxN <= 64, "one lane per row in the triangular solves");
    static_assert(kT == 256, "a 16 x 16 thread grid");
    const int t = threadIdx.x, ti = t >> 4, tj = t & 15;
    for (int k = 0; k < n; ++k) {
        const double d = A[k * n + k];
        if (!(d > 0.0 && isfinite(d))) return false;     // the same for every thread
        const double l = sqrt(d);
        for (int i = k + 1 + t; i < n; i += kT) A[k * n + i] = A[i * n + k] / l;
        if (t == 0) S.ldiag[k] = l;
        __syncthreads();
        const double *Lk = A + k * n;                    // L[i][k] = Lk[i], i > k
        for (int i = k + 1 + ti; i < n; i += 16) {
            const double lik = Lk[i];
            for (int j = k + 1 + tj; j <= i; j += 16) A[i * n + j] -= lik * Lk[j];
        }
        __syncthreads();
    }
    if (t < 64) {
        const int lane = t;
        // L y = b, with L[j][i] = A[i][j] for j > i
        for (int i = 0; i < n; ++i) {
            wave_lds_sync();
            const double yi = b[i] / S.ldiag[i];
            const int j = i + 1 + lane;
            if (j < n) b[j] -= A[i * n + j] * yi;
            if (lane == 0) x[i] = yi;
        }
        // L^T x = y, with L[i][j] = A[j][i] for j < i
        for (int i = n - 1; i >= 0; --i) {
            wave_lds_sync();
            const double xi = x[i] / S.ldiag[i];
            wave_lds_sync();                 // x[i] is read by every lane before it is rewritten
            if (lane == 0) x[i] = xi;
            for (int j = lane; j < i; j += 64) x[j] -= A[j * n + i] * xi;
        }
        wave_lds_sync();
        if (lane == 0) {
            int good = 1;
            for (int i = 0; i < n; ++i) good &= isfinite(x[i]) ? 1 : 0;
            S.ok = good;
        }
    }
    __syncthreads();
    return S.ok != 0;
}

// ---------------------------------------------------------------------------
// The LM bookkeeping (Marquardt 1963) after one evaluation, work-group 0.
// Damped system (H + mu D) delta = g with D = diag(max(H_ii, 1e-12 max
// H_ii)); a parameter on a bound whose gradient leaves the box is held for
// the trial; the trial point is clipped to the bounds; accept iff F
// decreases; gain-ratio damping (mu *= max(1/3, 1 - (2 rho - 1)^3) on accept,
// mu *= nu, nu *= 2 on reject); converged when an accepted step has
// max |delta_k| / scale_k < tol, or stalled once mu passes 1e8; the budget
// counts trials.  Sets S.finished when the fit is over; otherwise S.th_e
// holds the next trial point.
// ---------------------------------------------------------------------------

// Acceptance of the evaluated trial and the damping update (thread 0).
__device__ __forceinline__ void lm_accept(const Params &p, WGShared &S)
{
    const int m = S.m;
    S.finished = 0;
    if (S.phase == 0) {
        S.accept = 1;
        S.mu = p.lm_mu0;
        S.nu = 2.0;
        S.trials = 0;
        S.converged = 0;
        S.chi2_init = S.chi2e;
        S.phase = S.alt_pending ? 2 : 1;
        return;
    }
    if (S.phase == 2) {
        // the proposal against the simple start: the lower objective is the
        // start of LM; the damping is untouched
        double Fp = S.Fe;
        if (!isfinite(Fp)) Fp = INFINITY;
        S.accept = (Fp < S.F_c) ? 1 : 0;
        S.chose_prop = S.accept;
        if (S.accept) {
            S.chi2_init = S.chi2e;
            for (int i = 0; i < 4; ++i) S.th0[i] = S.th_e[i];
        }
        S.phase = 1;
        return;
    }
    double Ft = S.Fe;
    if (!isfinite(Ft)) Ft = INFINITY;
    S.accept = (Ft < S.F_c) ? 1 : 0;
    if (S.accept) {
        double step = 0.0;
        for (int j = 0; j < m; ++j) {
            const double *tn = S.th_e + 4 * j, *to = S.th_c + 4 * j;
            const double sa = fabs(tn[0]) > 1e-30 ? fabs(tn[0]) : 1e-30;
            double v;
            v = fabs(tn[0] - to[0]) / sa; step = v > step ? v : step;
            v = fabs(tn[1] - to[1]) / tn[3]; step = v > step ? v : step;
            v = fabs(tn[2] - to[2]) / tn[3]; step = v > step ? v : step;
            v = fabs(tn[3] - to[3]) / tn[3]; step = v > step ? v : step;
        }
        const double rho = S.pred > 0.0 ? (S.F_c - Ft) / S.pred : 1.0;
        const double tt = 2.0 * rho - 1.0;
        double f = 1.0 - tt * tt * tt;
        if (f < 1.0 / 3.0) f = 1.0 / 3.0;
        S.mu *= f;
        if (S.mu < 1e-12) S.mu = 1e-12;
        S.nu = 2.0;
        if (step < p.lm_tol) { S.converged = 1; S.finished = 1; }
    } else {
        S.mu *= S.nu;
        S.nu *= 2.0;
        if (S.mu > 1e8) { S.converged = 1; S.finished = 1; }
    }
}

// The damped solve for n = N <= 8 by thread 0 alone, the factor's lower
// triangle in registers: the same arithmetic as the work-group path below,
// with each Cholesky column scaled by one reciprocal square root.
template <int N>
__device__ __forceinline__ void lm_solve_small(int32_t lm_max_iter, WGShared &S, const double *Hc)
{
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) dmax = Hc[i * N + i] > dmax ? Hc[i * N + i] : dmax;
    double dd[N], rhs[N];
    bool fr[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double hii = Hc[i * N + i];
        dd[i] = hii < 1e-12 * dmax ? 1e-12 * dmax : hii;
        const double th = S.th_c[i], g = S.g_c[i];
        fr[i] = (th <= S.lo[i] && g <= 0.0) || (th >= S.hi[i] && g >= 0.0);
        rhs[i] = fr[i] ? 0.0 : g;
    }
    while (!S.finished) {
        if (S.trials >= lm_max_iter) { S.finished = 1; break; }
        S.trials++;
        const double mu = S.mu;
        double a[N][N];
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int k = 0; k <= i; ++k)
                a[i][k] = (fr[i] || fr[k]) ? (i == k ? 1.0 : 0.0)
                                           : Hc[i * N + k] + (i == k ? mu * dd[i] : 0.0);
        bool ok = true;
        double rinv[N];                  // 1 / L_kk
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double d = a[k][k];
            ok = ok && d > 0.0 && isfinite(d);
            const double r = ok ? 1.0 / sqrt(d) : 0.0;
            rinv[k] = r;
            a[k][k] = ok ? d * r : 1.0;
#pragma unroll
            for (int i = k + 1; i < N; ++i) a[i][k] *= r;
#pragma unroll
            for (int i = k + 1; i < N; ++i)
#pragma unroll
                for (int j = k + 1; j <= i; ++j) a[i][j] -= a[i][k] * a[j][k];
        }
        double x[N];
        if (ok) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double v = rhs[i];
#pragma unroll
                for (int j = 0; j < i; ++j) v -= a[i][j] * x[j];
                x[i] = v * rinv[i];
            }
#pragma unroll
            for (int i = N - 1; i >= 0; --i) {
                double v = x[i];
#pragma unroll
                for (int j = i + 1; j < N; ++j) v -= a[j][i] * x[j];
                x[i] = v * rinv[i];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) ok = ok && isfinite(x[i]);
        }
        if (ok) {
            double pred = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double v = S.th_c[i] + x[i];
                if (!(v >= S.lo[i])) v = S.lo[i];
                if (v > S.hi[i]) v = S.hi[i];
                S.th_e[i] = v;
                S.delta[i] = x[i];
                pred += x[i] * (rhs[i] + mu * dd[i] * x[i]);
            }
            S.pred = pred;
            break;
        }
        // not positive definite: treated as a rejected trial
        S.mu *= S.nu;
        S.nu *= 2.0;
        if (S.mu > 1e8) { S.converged = 1; S.finished = 1; }
    }
}

__device__ __forceinline__ void lm_step(const Params &p, WGShared &S, double *H2, double *A)
{
    const int t = threadIdx.x;
    const int n = S.n;
    if (t == 0) lm_accept(p, S);
    __syncthreads();
    if (S.accept) {
        // the evaluated point becomes the current one; its Gram matrix buffer
        // becomes the current buffer (no copy)
        if (t < n) { S.th_c[t] = S.th_e[t]; S.g_c[t] = S.ge[t]; }
        if (t == 0) {
            S.F_c = S.Fe; S.chi2_c = S.chi2e; S.npx_c = S.npx_e;
            S.hsel ^= 1;
        }
    }
    __syncthreads();
    if (S.phase == 2) {
        // the simple start is evaluated; the next evaluation is the proposal
        // start with the other members unchanged
        if (t < 4) {
            double v = S.alt[t];
            if (!(v >= S.lo[t])) v = S.lo[t];
            if (v > S.hi[t]) v = S.hi[t];
            S.th_e[t] = v;
        }
        if (t == 0) {
            S.alt_pending = 0;
            S.finished = 0;
        }
        __syncthreads();
        return;
    }
    const double *Hc = H2 + S.hsel * (kMaxN * kMaxN);
    if (n <= 8) {
        if (t == 0) {
            if (n == 4) lm_solve_small<4>(p.lm_max_iter, S, Hc);
            else lm_solve_small<8>(p.lm_max_iter, S, Hc);
        }
        __syncthreads();
        return;
    }
    for (;;) {
        __syncthreads();
        if (S.finished) break;
        if (t == 0) {
            if (S.trials >= p.lm_max_iter) S.finished = 1;
            else S.trials++;
        }
        if (t < 64) {
            // the largest diagonal entry: a max over the lanes of wave 0
            double dmax = t < n ? Hc[t * n + t] : 0.0;
            for (int off = 32; off > 0; off >>= 1) {
                const double o = __shfl_xor(dmax, off, 64);
                dmax = o > dmax ? o : dmax;
            }
            if (t < n) {
                const double d = Hc[t * n + t];
                S.dd[t] = d < 1e-12 * dmax ? 1e-12 * dmax : d;
                const double th = S.th_c[t], g = S.g_c[t];
                S.frozen[t] = ((th <= S.lo[t] && g <= 0.0) || (th >= S.hi[t] && g >= 0.0)) ? 1 : 0;
                S.rhs[t] = S.frozen[t] ? 0.0 : g;
            }
        }
        __syncthreads();
        if (S.finished) break;
        const double mu = S.mu;
        for (int i = t >> 4; i < n; i += 16) {
            for (int k = t & 15; k < n; k += 16) {
                double v;
                if (S.frozen[i] || S.frozen[k]) v = (i == k) ? 1.0 : 0.0;
                else v = Hc[i * n + k] + (i == k ? mu * S.dd[i] : 0.0);
                A[i * n + k] = v;
            }
        }
        if (t < n) S.rhs_copy[t] = S.rhs[t];
        __syncthreads();
        const bool ok = chol_solve(S, A, n, S.rhs_copy, S.delta);
        if (ok) {
            if (t < n) {
                double v = S.th_c[t] + S.delta[t];
                if (!(v >= S.lo[t])) v = S.lo[t];
                if (v > S.hi[t]) v = S.hi[t];
                S.th_e[t] = v;
            }
            if (t == 0) {
                double pred = 0.0;
                for (int i = 0; i < n; ++i)
                    pred += S.delta[i] * (S.rhs[i] + mu * S.dd[i] * S.delta[i]);
                S.pred = pred;
            }
            __syncthreads();
            break;
        }
        if (t == 0) {       // not positive definite: treated as a rejected trial
            S.mu *= S.nu;
            S.nu *= 2.0;
            if (S.mu > 1e8) { S.converged = 1; S.finished = 1; }
        }
    }
    __syncthreads();
}

// Commit and the residual-update plan, work-group 0.  The loop gain (Sect. 3)
// scales every change the fit makes to the model image: the new component
// joins with gain times its fitted amplitude at its fitted centre and width,
// and each old member moves the fraction gain of the way from its stored
// parameters to its refit.  A new component whose fitted amplitude is zero
// (held on its sign bound: the old members explain the peak) models no
// emission and is not added to the list.
__device__ __forceinline__ void commit(const Params &p, WGShared &S)
{
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int m = S.m;
    if (t == 0) {
        const int64_t L = st->L, k = st->k;
        const int trials = S.trials_total + S.trials;
        st->n_active = m;
        st->lm_iters = trials;
        st->converged = S.converged;
        st->used_fallback = S.used_fallback;
        st->chi2_init = S.chi2_init;
        st->chi2_final = S.chi2_c;
        st->fit_px = S.npx_c;
        st->sum_trials += (unsigned long long)trials;
        st->not_converged += S.converged ? 0ull : 1ull;
        st->fallbacks += (unsigned long long)S.used_fallback;
        st->init_source = S.use_prop ? st->have_proposal : (S.use_smooth ? 3 : 0);
        // a fallback follows only a fit that started from the proposal
        st->start_prop = (S.chose_prop || S.used_fallback) ? 1 : 0;
        for (int i = 0; i < 4; ++i)
            st->init[i] = S.use_prop ? st->proposal[i] : (S.use_smooth ? S.t0[i] : 0.0);
        st->have_proposal = 0;
        if (p.smooth) {
            // Sect. 3's switch: the simple values next time when the new
            // component's fitted area fell below 5 % of its start's area
            const double s0 = S.t0[3], s1 = S.th_c[3], wb = st->omega_b;
            const bool shrank = p.sm.switch_area
                                    ? __dsub_rn(__dmul_rn(s1, s1), __dmul_rn(wb, wb)) <
                                          __dmul_rn(0.05, __dsub_rn(__dmul_rn(s0, s0), __dmul_rn(wb, wb)))
                                    : __dmul_rn(s1, s1) < __dmul_rn(0.05, __dmul_rn(s0, s0));
            st->smooth_now = shrank ? 0 : 1;
            st->smooth_ready = 0;
            st->sum_smoothed += S.use_smooth ? 1ull : 0ull;
        }
        if (p.rec_cap > 0 && st->rec_n < p.rec_cap) {
            // the training pair of this iteration: the patch is already in place
            const int64_t n = st->rec_n;
            const int64_t r0 = S.idx / p.W, c0 = S.idx % p.W;
            float *tg = p.rec_target + 4 * n;
            tg[0] = (float)(S.th_c[0] / S.peak);
            tg[1] = (float)log(S.th_c[3] / st->omega_b);
            tg[2] = (float)(S.th_c[1] - (double)c0);
            tg[3] = (float)(S.th_c[2] - (double)r0);
            p.rec_flag[n] = S.converged | (S.used_fallback << 1) | (st->init_source << 2);
            st->rec_n = n + 1;
        }
        int nr = 0;
        int32_t bb[4] = {INT32_MAX, -1, INT32_MAX, -1};
        auto add_rect = [&](double a, double x, double y, double s, float sign) {
            Rect &R = st->rects[nr++];
            int32_t w[4];
            make_window(x, y, halfwidth(s, p.window_sigmas), p.H, p.W, w);
            R.r0 = w[0]; R.r1 = w[1]; R.c0 = w[2]; R.c1 = w[3];
            R.a = a; R.x = x; R.y = y; R.s = s; R.sign = sign;
            bb[0] = w[0] < bb[0] ? w[0] : bb[0];
            bb[1] = w[1] > bb[1] ? w[1] : bb[1];
            bb[2] = w[2] < bb[2] ? w[2] : bb[2];
            bb[3] = w[3] > bb[3] ? w[3] : bb[3];
        };
        for (int j = 1; j < m; ++j) {
            const int64_t cj = S.members[j];
            const double *to = S.th_old + 4 * j, *tn = S.th_c + 4 * j;
            double tc[4];
            // t + gain (t* - t), each operation rounded on its own
            for (int q = 0; q < 4; ++q)
                tc[q] = __dadd_rn(to[q], __dmul_rn(p.gain, __dsub_rn(tn[q], to[q])));
            add_rect(to[0], to[1], to[2], to[3], +1.0f);
            add_rect(tc[0], tc[1], tc[2], tc[3], -1.0f);
            p.ca[cj] = tc[0]; p.cx[cj] = tc[1]; p.cy[cj] = tc[2]; p.cs[cj] = tc[3];
            p.c_updated[cj] = k;
        }
        const bool added = S.th_c[0] != 0.0;
        if (added) {
            const double anew = __dmul_rn(p.gain, S.th_c[0]);
            add_rect(anew, S.th_c[1], S.th_c[2], S.th_c[3], -1.0f);
            p.ca[L] = anew; p.cx[L] = S.th_c[1]; p.cy[L] = S.th_c[2]; p.cs[L] = S.th_c[3];
            p.c_added[L] = k;
            p.c_updated[L] = k;
        }
        st->added = added ? 1 : 0;
        st->not_added += added ? 0ull : 1ull;
        st->n_rects = nr;
        if (nr == 0) { bb[0] = 0; bb[1] = -1; bb[2] = 0; bb[3] = -1; }
        st->bb[0] = bb[0]; st->bb[1] = bb[1]; st->bb[2] = bb[2]; st->bb[3] = bb[3];
        st->L = added ? L + 1 : L;
        st->k = k + 1;
        st->fit_ready = 1;
    }
    if (t < m) st->members[t] = S.members[t];
    if (t < 4 * m) {
        st->theta0[t] = S.th0[t];
        st->theta[t] = S.th_c[t];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------

// Evaluate this work-group's tiles of the trial prepared in S into row.
__device__ __forceinline__ void evaluate_row(const Params &p, WGShared &S, float *tile, double *red, int64_t tile0,
                             int64_t stride, double *row)
{
    if (S.m == 1) evaluate_tiles_reg<1>(p, S, tile0, stride, row, tile);
    else if (S.m == 2) evaluate_tiles_reg<2>(p, S, tile0, stride, row, tile);
    else if (S.m <= 3) evaluate_tiles_mfma<1>(p, S, tile, tile0, stride, row);
    else if (S.m <= 7) evaluate_tiles_mfma<2>(p, S, tile, tile0, stride, row);
    else if (S.m <= 11) evaluate_tiles_mfma<3>(p, S, tile, tile0, stride, row);
    else if (S.m <= 15) evaluate_tiles_mfma<4>(p, S, tile, tile0, stride, row);
    else evaluate_tiles(p, S, tile, red, tile0, stride, row);
}

// Work-groups of a shared trial: at least min_tiles tiles each.
__device__ inline int eval_groups(int64_t ntiles, int nwg, int min_tiles)
{
    const int64_t want = (ntiles + min_tiles - 1) / min_tiles;
    return (int)(want < nwg ? want : nwg);
}

// Arrival of one work-group after a shared trial (every work-group, every
// round): the last of a group sums the group's evaluated rows in order into
// the group row and arrives at the top counter.
__device__ __forceinline__ void arrive(const Params &p, FitGlobal *G, WGShared &S, int wg, int nwg,
                                       int geff, bool acquire = true)
{
    const int t = threadIdx.x;
    const int gs = p.group;
    const int grp = wg / gs;
    const int gsize = (grp + 1) * gs < nwg ? gs : nwg - grp * gs;
    const int ng_eval = (geff + gs - 1) / gs;
    __syncthreads();
    if (t == 0) {
        // the group rows are read with atomic loads, so the acquire is optional
        const unsigned prev =
            acquire ? __hip_atomic_fetch_add(&G->arrive_g[grp], 1u, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT)
                    : __hip_atomic_fetch_add(&G->arrive_g[grp], 1u, __ATOMIC_RELEASE,
                                             __HIP_MEMORY_SCOPE_AGENT);
        S.last = (prev == (unsigned)gsize - 1u) ? 1 : 0;
        if (S.last)
            __hip_atomic_store(&G->arrive_g[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!S.last) return;
    const int r0 = grp * gs, r1 = (r0 + gs < geff) ? r0 + gs : geff;
    if (ng_eval > 1 && r0 < r1) sum_rows(p, S.n, r0, r1, nwg + grp);
    __syncthreads();
    if (t == 0) __hip_atomic_fetch_add(&G->top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Flat arrival of a shared trial of at most eight parameters (k_fit only):
// every work-group, work-group 0 included, adds itself to its group's counter
// with one release and leaves; no group sums its rows.  Work-group 0 waits for
// every group (flat_wait), resets the counters, and sums all the evaluated rows
// itself (reduce_flat), in the association of the two-level sums: rows in
// order within a group of p.group, then the groups in order.
constexpr int kFlatMaxN = 8;
static_assert(sizeof(double) * ((kFlatMaxN + 1) * (kFlatMaxN + 2) / 2 + 3) * kMaxGroups <=
                  kTileBytes, "group sums of the flat reduction in the tile buffer");
__device__ __forceinline__ void arrive_flat(FitGlobal *G, int wg, int gs)
{
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&G->arrive_g[wg / gs], 1u, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Work-group 0: lane g of wave 0 polls group g's counter until the group is
// complete (every group of the grid, evaluating or not, so that no late
// arrival can count toward the next trial), then clears it.  Bounded in time.
__device__ __forceinline__ bool flat_wait(FitGlobal *G, WGShared &S, int nwg, int gs,
                                          unsigned long long limit)
{
    const int t = threadIdx.x;
    const int ngroups = (nwg + gs - 1) / gs;
    if (t < 64) {
        const int g = t;
        const bool live = g < ngroups;
        const unsigned need = live ? (unsigned)((g + 1) * gs < nwg ? gs : nwg - g * gs) : 0u;
        const unsigned long long t0 = now_ticks();
        bool ok = true;
        for (;;) {
            const unsigned v = live ? __hip_atomic_load(&G->arrive_g[g], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : 0u;
            if (__all(v >= need)) break;
            if (now_ticks() - t0 > limit) { ok = false; break; }
            __builtin_amdgcn_s_sleep(kPollSleep);
        }
        if (live) __hip_atomic_store(&G->arrive_g[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t == 0) S.abort = ok ? 0 : 1;
    }
    __syncthreads();
    return S.abort == 0;
}

// The evaluated rows 0 .. geff-1 summed into He, S.ge, S.Fe, S.chi2e, S.npx_e
// with the two-level association; `scratch` holds the group sums
// ((n_out + 3) x groups doubles, LDS).
__device__ __forceinline__ void reduce_flat(const Params &p, WGShared &S, int geff, int gs,
                                            double *He, double *scratch)
{
    const int n = S.n;
    const int n_out = (n + 1) * (n + 2) / 2, nv = n_out + 3;
    const int ng = (geff + gs - 1) / gs;
    for (int e = threadIdx.x; e < nv * ng; e += kT) {
        const int o = e % nv, g = e / nv;
        const int r0 = g * gs, r1 = r0 + gs < geff ? r0 + gs : geff;
        scratch[g * nv + o] = sum_column(p, r0, r1, o);
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nv; o += kT) {
        double v = scratch[o];
        for (int g = 1; g < ng; ++g) v += scratch[g * nv + o];
        if (o >= n_out) {
            if (o == n_out) S.Fe = v;
            else if (o == n_out + 1) S.chi2e = v;
            else S.npx_e = (int64_t)v;
            continue;
        }
        int i, k;
        out_pair(o, n, i, k);
        if (i < n && k < n) { He[i * n + k] = v; He[k * n + i] = v; }
        else if (i < n) S.ge[i] = v;
    }
    __syncthreads();
}

// The peak and the stop test (Sect. 2 steps 1 and 4) of one fit, thread 0 of
// the leading work-group: sets S.idx, S.peak, S.stop and the fit's
// bookkeeping.  `abort` reports a wait that ran out before it.
__device__ __forceinline__ void fit_begin(const Params &p, WGShared &S, bool abort)
{
    DevState *st = p.st;
    atomicAdd(&st->prof[kPFits], 1ull);
    st->fit_ready = 0;
    const unsigned long long key = S.key;
    int64_t idx = st->forced_idx >= 0
                      ? st->forced_idx
                      : (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    const bool bad_idx = (st->forced_idx < 0 && key == 0ull) || idx < 0 || idx >= p.H * p.W;
    st->forced_idx = -1;
    S.stop = 0;
    if (abort) S.stop = ASP_ERR_DEVICE;
    else if (bad_idx) S.stop = ASP_ERR_STATE;
    if (bad_idx) idx = 0;
    const float v = p.R[idx];
    if (S.stop == 0) {
        if (fabs((double)v) < p.threshold) S.stop = ASP_STOP_THRESHOLD;
        else if (st->k >= p.max_iter) S.stop = ASP_STOP_MAXITER;
        else if (st->L >= p.cap) S.stop = ASP_ERR_CAPACITY;
    }
    st->idx = idx;
    st->peak = v;
    S.idx = idx;
    S.peak = (double)v;
    S.pass = 0;
    S.trials_total = 0;
    S.used_fallback = 0;
    S.use_prop = (p.use_proposal && st->have_proposal) ? 1 : 0;
    S.use_smooth = (p.smooth && !S.use_prop && st->smooth_now && st->smooth_ready) ? 1 : 0;
    if (S.stop) st->stop = S.stop;
}

// One evaluation of the trial at S.th_e (old members at S.th_old) by the
// leading work-group: F, chi2, the pixel count and [J r]^T [J r] reduced into
// S.Fe, S.chi2e, S.npx_e, S.ge and the Gram buffer H2 + (1 - S.hsel) n^2.  A
// trial larger than p.solo_tiles tiles is published (with G->cmd = cmd when
// cmd != 0) and shared by the nwg work-groups.  Returns false when a wait ran
// out; the context is then marked with ASP_ERR_DEVICE.
__device__ __forceinline__ bool trial_eval(const Params &p, FitGlobal *G, WGShared &S, float *tile,
                                           double *red, double *H2, int nwg, int cmd)
{
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int ngroups = (nwg + p.group - 1) / p.group;
    prepare(p, S, S.m, S.th_e, S.th_old);
    const int64_t ntiles = (S.pref[S.m] + kT - 1) / kT;
    lap(p, S, kPPrepare);
    double *He = H2 + (1 - S.hsel) * (kMaxN * kMaxN);   // the trial's buffer
    if (ntiles <= p.solo_tiles) {
        // small: the leading work-group alone, no publication
        if (t == 0) atomicAdd(&p.st->prof[kPSoloTrials], 1ull);
        evaluate_row(p, S, tile, red, 0, 1, p.partials);
        lap(p, S, kPEval);
        reduce_partials(p, S, 0, 1, He);
        lap(p, S, kPReduce);
        if (t == 0) atomicAdd(&p.st->prof[kPSoloPx], (unsigned long long)S.npx_e);
        return true;
    }
    // large: every work-group takes a share
    const int geff = eval_groups(ntiles, nwg, p.min_tiles);
    const int ng_eval = (geff + p.group - 1) / p.group;
    if (t < S.n) G->th_e[t] = S.th_e[t];
    if (t == 0 && cmd) G->cmd = cmd;
    publish(G);
    evaluate_row(p, S, tile, red, 0, geff, p.partials);
    lap(p, S, kPEval);
    if (cmd == 0 && S.n <= kFlatMaxN) {
        arrive_flat(G, 0, p.group);
        lap(p, S, kPArrive);
        const bool ok = flat_wait(G, S, nwg, p.group, p.spin_ticks);
        lap(p, S, kPWait);
        if (!ok) {
            if (t == 0) st->stop = ASP_ERR_DEVICE;
            __syncthreads();
            return false;
        }
        reduce_flat(p, S, geff, p.group, He, reinterpret_cast<double *>(tile));
        lap(p, S, kPReduce);
        return true;
    }
    arrive(p, G, S, 0, nwg, geff, false);
    lap(p, S, kPArrive);
    if (t == 0) {
        // the rows are read with atomic loads: no acquire
        S.abort = spin_until(&G->top, (unsigned)ngroups, p.spin_ticks, false) ? 0 : 1;
        __hip_atomic_store(&G->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    lap(p, S, kPWait);
    __syncthreads();
    if (S.abort) {
        if (t == 0) st->stop = ASP_ERR_DEVICE;
        __syncthreads();
        return false;
    }
    if (ng_eval > 1) reduce_partials(p, S, nwg, nwg + ng_eval, He);
    else reduce_partials(p, S, 0, geff, He);
    lap(p, S, kPReduce);
    return true;
}

// Start values, active set, the LM trials and the commit of one fit, by the
// leading work-group (share 0 of nwg).  A trial larger than p.solo_tiles tiles
// is published (with G->cmd = cmd when cmd != 0) and shared by the nwg
// work-groups.  Returns false when a wait ran out; the context is then marked
// with ASP_ERR_DEVICE.
__device__ __forceinline__ bool fit_trials(const Params &p, FitGlobal *G, WGShared &S, float *tile,
                                           double *red, double *A, double *H2,
                                           int nwg, int cmd)
{
    DevState *st = p.st;
    const int t = threadIdx.x;
    mark(S);
    if (t == 0) S.tfit = S.tmark;
    setup_fit(p, G, S, S.use_prop != 0);
    lap(p, S, kPSetup);
    for (;;) {
        if (!trial_eval(p, G, S, tile, red, H2, nwg, cmd)) return false;
        lm_step(p, S, H2, A);
        lap(p, S, kPLmStep);
        if (t == 0) {
            const unsigned long long npx = (unsigned long long)S.npx_e;
            st->sum_eval_px += npx;
            st->sum_gram_flops += npx * (unsigned long long)((S.n + 1) * (S.n + 2));
            atomicAdd(&st->prof[kPTrials], 1ull);
            atomicAdd(&st->prof[kPEvalPx], npx);
        }
        if (!S.finished) continue;
        if (S.use_prop && S.chose_prop && S.pass == 0 && (!S.converged || S.th_c[0] == 0.0)) {
            // LM started from the proposal and did not converge, or converged
            // to a new component of zero amplitude (which can leave the model
            // unchanged, so that the same peak and proposal come back): the
            // simple values instead
            if (t == 0) {
                S.trials_total += S.trials;
                S.used_fallback = 1;
                S.pass = 1;
            }
            __syncthreads();
            setup_fit(p, G, S, false);
            continue;
        }
        mark(S);
        commit(p, S);
        lap(p, S, kPCommit);
        if (t == 0) {
            const int m = S.m;
            st->fits_m[m] += 1ull;
            st->trials_m[m] += (unsigned long long)(S.trials_total + S.trials);
            st->ticks_m[m] += now_ticks() - S.tfit;
        }
        return true;
    }
}

__global__ __launch_bounds__(kT) void k_fit(Params p)
{
    extern __shared__ __align__(16) unsigned char lds[];
    float *tile = reinterpret_cast<float *>(lds);
    double *A = reinterpret_cast<double *>(lds);               // shares the tile buffer
    double *H2 = reinterpret_cast<double *>(lds + kTileBytes);   // two Gram buffers
    __shared__ WGShared S;
    __shared__ double red[kT];
    FitGlobal *G = p.fg;
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int wg = blockIdx.x, nwg = gridDim.x;

    // Nothing writes the stop flag (or the evaluation request) before every
    // work-group has checked in, so all of them agree here.
    if (st->stop && st->diag_m == 0) return;

    mark(S);
    // Check in: every work-group reads the generation before work-group 0 may
    // publish.
    if (t == 0) {
        S.gen = __hip_atomic_load(&G->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.abort = 0;
        __hip_atomic_fetch_add(&G->top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();

    if (wg != 0) {
        // Workers: evaluate the shared trials work-group 0 publishes.
        // The residual does not change inside this kernel and everything
        // published is read with atomic loads, so the workers need no acquire
        // fence: their L2 keeps the residual's lines from trial to trial.
        for (;;) {
            if (!wait_publish(G, S, p.spin_ticks, false)) {
                if (t == 0) st->stop = ASP_ERR_DEVICE;
                return;
            }
            if (t == 0) {
                S.done = ld_shared(&G->done);
                S.cmd = ld_shared(&G->m);
            }
            __syncthreads();
            if (S.done) {
                if (S.done == 2) {
                    // the committed plan was written by work-group 0 with plain
                    // stores: acquire before reading it
                    if (t == 0) acquire_fence();
                    __syncthreads();
                    update_tiles(p, wg, nwg, tile);
                }
                return;
            }
            prepare(p, S, S.cmd, G->th_e, G->th_old, true);
            const int64_t ntiles = (S.pref[S.m] + kT - 1) / kT;
            const int geff = eval_groups(ntiles, nwg, p.min_tiles);
            if (wg < geff)
                evaluate_row(p, S, tile, red, wg, geff, p.partials + (int64_t)wg * kPartStride);
            if (S.n <= kFlatMaxN) arrive_flat(G, wg, p.group);
            else arrive(p, G, S, wg, nwg, geff, false);
        }
    }

    // Work-group 0 drives the fit.
    if (t == 0) {
        S.abort = spin_until(&G->top, (unsigned)nwg, p.spin_ticks) ? 0 : 1;
        __hip_atomic_store(&G->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lap(p, S, kPCheckin);
    }
    __syncthreads();
    if (st->diag_m > 0) {
        // one evaluation of a given trial (asp_eval_trial): no peak, no LM
        // step, no commit
        if (t == 0) {
            S.m = st->diag_m;
            S.n = 4 * S.m;
            S.hsel = 0;
            G->m = S.m;
            G->n = S.n;
            G->done = 0;
        }
        __syncthreads();
        if (t < S.n) {
            S.th_e[t] = st->diag_theta[t];
            S.th_old[t] = st->diag_stored[t];
            G->th_old[t] = S.th_old[t];
        }
        __syncthreads();
        const bool ok = !S.abort && trial_eval(p, G, S, tile, red, H2, nwg, 0);
        const int n = S.n;
        double *o = st->diag_out;
        if (ok) {
            const double *He = H2 + kMaxN * kMaxN;        // 1 - hsel
            for (int e = t; e < n * n; e += kT) o[e] = He[e];
            if (t < n) o[n * n + t] = S.ge[t];
            if (t == 0) {
                o[n * n + n] = S.Fe;
                o[n * n + n + 1] = S.chi2e;
                o[n * n + n + 2] = (double)S.npx_e;
            }
        }
        if (t == 0) {
            if (!ok) st->stop = ASP_ERR_DEVICE;
            st->diag_m = 0;
            G->done = 1;
        }
        publish(G);
        return;
    }
    collect_peak_key(st, true, &S.key);
    if (t == 0) {
        fit_begin(p, S, S.abort != 0);
        // workers read this only after a publication of this fit
        G->done = S.stop ? 1 : 0;
    }
    __syncthreads();
    if (!S.stop) {
        const bool committed = fit_trials(p, G, S, tile, red, A, H2, nwg, 0);
        // with fuse_update every work-group takes its tiles of the update
        // (Sect. 2 step 3) after this publication; the end of the kernel is
        // the barrier before the next iteration reads R
        if (t == 0) {
            S.upd = committed && p.fuse_update ? 1 : 0;
            G->done = S.upd ? 2 : 1;
        }
    }
    publish(G);
    if (!S.stop && S.upd) update_tiles(p, 0, nwg, tile);
}

// ===========================================================================
// Batched fields: one persistent launch for many independent fields.
//
// The work-groups form teams of T.  Work-groups are dealt to the 8 XCDs round
// robin, so a team is made of work-groups with equal blockIdx % 8: one XCD,
// one L2 for the team's field.  A team takes fields from a queue, largest
// first, and runs each field's minor cycle for up to n_iter iterations:
// rank 0 leads as work-group 0 of k_fit does and the others follow its
// commands -- a share of the peak search, a share of an LM trial, a share of
// the residual update, or exit.  Every command is acknowledged by every member
// before the next one is published; every wait is bounded.
// ===========================================================================

enum { kCmdPeak = 1, kCmdEval = 2, kCmdUpdate = 3, kCmdExit = 4 };

// The field's parameters with the team's exchange buffers and the batch's
// tile thresholds (thread 0 writes, the work-group reads after the barrier).
__device__ __forceinline__ void load_field(const BatchArgs &b, int f, FitGlobal *G, double *parts,
                                           Params &P)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        P = b.fields[f];
        P.fg = G;
        P.partials = parts;
        P.solo_tiles = b.team_size == 1 ? 0x7FFFFFFF : b.solo_tiles;
        P.min_tiles = b.min_tiles;
        P.group = kGroup;
    }
    __syncthreads();
}

// The leader's wait for the team's arrivals; false when it ran out.
__device__ __forceinline__ bool team_wait(FitGlobal *G, WGShared &S, int ngroups,
                                          unsigned long long limit)
{
    if (threadIdx.x == 0) {
        S.abort = spin_until(&G->top, (unsigned)ngroups, limit) ? 0 : 1;
        __hip_atomic_store(&G->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return S.abort == 0;
}

__global__ __launch_bounds__(kT) void k_batch(BatchArgs b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    float *tile = reinterpret_cast<float *>(lds);
    double *A = reinterpret_cast<double *>(lds);
    double *H2 = reinterpret_cast<double *>(lds + kTileBytes);   // two Gram buffers
    __shared__ WGShared S;
    __shared__ double red[kT];
    __shared__ Params P;
    __shared__ int32_t cur_field;
    const int t = threadIdx.x;
    const int T = b.team_size;
    const int per_xcd = (int)gridDim.x / 8;
    const int xcd = (int)blockIdx.x % 8, slot = (int)blockIdx.x / 8;
    const int team = xcd * (per_xcd / T) + slot / T;
    const int rank = slot % T;
    const int ngroups = (T + kGroup - 1) / kGroup;
    FitGlobal *G = b.fg + team;
    double *parts = b.partials + (int64_t)team * (T + ngroups) * kPartStride;

    // check in: every follower reads the generation before the leader publishes
    if (t == 0) {
        S.gen = __hip_atomic_load(&G->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.abort = 0;
        cur_field = -1;
        if (rank != 0)
            __hip_atomic_fetch_add(&G->top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();

    if (rank != 0) {
        for (;;) {
            if (!wait_publish(G, S, b.spin_ticks, true, true)) return;  // the leader marks its field
            if (t == 0) {
                S.cmd = G->cmd;
                S.fld = G->field;
            }
            __syncthreads();
            const int cmd = S.cmd;
            if (cmd == kCmdExit || S.fld < 0 || S.fld >= b.n_fields) return;
            if (S.fld != cur_field) {
                load_field(b, S.fld, G, parts, P);
                if (t == 0) cur_field = S.fld;
                __syncthreads();
            }
            int geff = 0;
            if (cmd == kCmdPeak) {
                peak_scan(P.R, P.H * P.W, (uint32_t)rank, (uint32_t)T, P.st->peak_keys);
            } else if (cmd == kCmdUpdate) {
                update_tiles<1>(P, rank, T, tile);
            } else if (cmd == kCmdEval) {
                prepare(P, S, ld_shared(&G->m), G->th_e, G->th_old, true);
                const int64_t ntiles = (S.pref[S.m] + kT - 1) / kT;
                geff = eval_groups(ntiles, T, P.min_tiles);
                if (rank < geff)
                    evaluate_row(P, S, tile, red, rank, geff,
                                 P.partials + (int64_t)rank * kPartStride);
            }
            arrive(P, G, S, rank, T, geff);
        }
    }

    // the leader
    if (t == 0) {
        if (T > 1) S.abort = spin_until(&G->top, (unsigned)(T - 1), b.spin_ticks) ? 0 : 1;
        __hip_atomic_store(&G->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    bool ok = S.abort == 0;
    while (ok) {
        if (t == 0) {
            const unsigned q = atomicAdd(b.queue, 1u);
            S.fld = q < (unsigned)b.n_fields ? b.order[q] : -1;
        }
        __syncthreads();
        if (S.fld < 0) break;
        load_field(b, S.fld, G, parts, P);
        if (t == 0) {
            cur_field = S.fld;
            G->field = S.fld;
            S.k_target = P.st->k + b.n_iter;
        }
        for (;;) {
            if (t == 0) {
                S.go = (P.st->stop == 0 && P.st->k < S.k_target) ? 1 : 0;
                // one heartbeat per iteration: the followers' waits restart
                __hip_atomic_fetch_add(&G->beat, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            if (!S.go) break;
            // the peak of |R| (Sect. 2 step 1)
            const int64_t npx = P.H * P.W;
            if (T == 1 || npx <= b.solo_peak_px) {
                peak_scan(P.R, npx, 0u, 1u, P.st->peak_keys);
            } else {
                if (t == 0) G->cmd = kCmdPeak;
                publish(G);
                peak_scan(P.R, npx, 0u, (uint32_t)T, P.st->peak_keys);
                arrive(P, G, S, 0, T, 0);
                if (!team_wait(G, S, ngroups, b.spin_ticks)) { ok = false; break; }
            }
            __syncthreads();
            // the stop test and the fit (Sect. 2 step 4; Sect. 3)
            collect_peak_key(P.st, true, &S.key);
            if (t == 0) fit_begin(P, S, false);
            __syncthreads();
            if (S.stop) break;
            if (!fit_trials(P, G, S, tile, red, A, H2, T, kCmdEval)) { ok = false; break; }
            // the residual update (Sect. 2 step 3)
            if (t == 0) {
                const int32_t *bb = P.st->bb;
                S.upx = (int64_t)(bb[1] - bb[0] + 1) * (int64_t)(bb[3] - bb[2] + 1);
            }
            __syncthreads();
            if (T == 1 || S.upx <= b.solo_update_px) {
                update_tiles<1>(P, 0, 1, tile);
            } else {
                if (t == 0) G->cmd = kCmdUpdate;
                publish(G);
                update_tiles<1>(P, 0, T, tile);
                arrive(P, G, S, 0, T, 0);
                if (!team_wait(G, S, ngroups, b.spin_ticks)) { ok = false; break; }
            }
        }
    }
    if (!ok && t == 0 && cur_field >= 0) P.st->stop = ASP_ERR_DEVICE;
    __syncthreads();
    if (T > 1) {
        if (t == 0) G->cmd = kCmdExit;
        publish(G);
    }
}

__global__ void k_batch_reset(unsigned int *queue) { *queue = 0u; }

hipError_t fit_kernel_setup()
{
    hipError_t e = hipFuncSetAttribute((const void *)k_fit,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFitLds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kFitLds);
}

// A kernel whose work-groups wait for each other must have all of them
// resident at once.  A private segment (scratch) breaks that guarantee: the
// waves of a dispatch can be held back until scratch is free.
static bool no_private_segment(const void *kernel)
{
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, kernel) != hipSuccess) return false;
    return a.localSizeBytes == 0;
}

int batch_grid_size(int device)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    if (!no_private_segment((const void *)k_batch)) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch, kT,
                                                     kFitLds) != hipSuccess || per_cu < 1)
        return 0;
    const int grid = (cus * per_cu / 8) * 8;      // whole XCD rows
    return grid <= cus * per_cu ? grid : 0;
}

hipError_t launch_batch(const BatchArgs &b, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, b.queue);
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kT), kFitLds, s, b);
    return hipGetLastError();
}

int fit_grid_size(int device)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    if (!no_private_segment((const void *)k_fit)) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fit, kT, kFitLds) !=
            hipSuccess || per_cu < 1)
        return 0;
    int g = cus * per_cu;
    if (g > kGroup * kMaxGroups) g = kGroup * kMaxGroups;
    return g;
}

hipError_t launch_fit(const Params &p, hipStream_t s)
{
    void *args[] = {(void *)&p};
    return hipLaunchCooperativeKernel((const void *)k_fit, dim3(p.fit_grid), dim3(kT), args,
                                      kFitLds, s);
}

}  // namespace asp
