// The active-set Levenberg-Marquardt fit of the Asp-Clean2016 minor cycle
// (Zhang, Bhatnagar, Rau & Zhang 2016, Sect. 3, Eq. 4) spread over the whole
// GPU.
//
// One cooperative launch, one work-group per CU.  Work-group 0 takes the
// peak, applies the stop test (Sect. 2 step 4), forms the start values (the
// simple initial values of Sect. 3, or a clamped proposal) and selects the
// active set.  Every LM trial then evaluates
//     F(theta) = sum_{U(theta)} M (M - 2 D),   H = J^T J,   g = J^T (D - M)
// over U(theta), the union of the members' windows at theta (a truncated
// Gaussian is zero outside its window, so this is the whole-image objective
// of Eq. 4 up to a constant).  D is the residual with the old members'
// stored Gaussians added back.  The 256-pixel tiles of U are dealt to the
// work-groups.  Per pixel, D, M, the residual r = D - M and the objective
// term M (M - 2D) are formed in FP64 (r is a small difference of O(1) terms);
// J (from the same values) and r go to FP32 for the augmented Gram matrix
// [J r]^T [J r], accumulated with Kahan compensation, while F and chi2 are
// accumulated in FP64.  Each work-group writes an FP64 partial; the last
// work-group to arrive sums the partials in
// work-group order, solves the damped normal equations by Cholesky in FP64,
// runs the LM bookkeeping and publishes the next trial point.  The work-group
// that finishes the fit commits it (loop gain on the new component, refits
// replace the old members) and writes the residual-update plan.
//
// Every wait is bounded; a wait that runs out marks the context with
// ASP_ERR_DEVICE and every work-group leaves.
#include <math.h>

#include "asp_device.h"

namespace asp {

constexpr int kT = kFitThreads;
constexpr int kOwnMax = (kNOutMax + kT - 1) / kT;
constexpr size_t kFitLds =
    sizeof(float) * kT * kTileStride + sizeof(double) * (2 * kMaxN * kMaxN + kT);
constexpr long kSpinLimit = 1L << 22;

struct WGShared {
    int32_t win[kMaxM][4], wold[kMaxM][4];
    int64_t pref[kMaxM + 1];
    double mx[kMaxM], my[kMaxM], mamp[kMaxM], minv2[kMaxM], minvs2[kMaxM], minvs3[kMaxM];
    double ox[kMaxM], oy[kMaxM], oamp[kMaxM], oinv2[kMaxM];
    int32_t m, n;
    double ge[kMaxN], Fe, chi2e;
    int64_t npx_e;
    double dd[kMaxN], rhs[kMaxN], rhs_copy[kMaxN], delta[kMaxN], th_t[kMaxN];
    int32_t frozen[kMaxN];
    uint32_t mask[kT];
    double t0[4];
    int32_t members[kMaxM];
    int32_t nch, sel_done;
    unsigned int gen;
    int32_t last, abort, done, ok, finished, accept, stop;
};

// ---------------------------------------------------------------------------
// Synchronisation between work-groups.
// ---------------------------------------------------------------------------

__device__ bool wait_publish(FitGlobal *G, WGShared &S)
{
    if (threadIdx.x == 0) {
        unsigned int now = S.gen;
        // relaxed polling (no cache invalidation per poll); the fence below
        // is the acquire
        for (long it = 0; it < kSpinLimit; ++it) {
            now = __hip_atomic_load(&G->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (now != S.gen) break;
            __builtin_amdgcn_s_sleep(2);
        }
        S.abort = (now == S.gen) ? 1 : 0;
        S.gen = now;
    }
    __syncthreads();
    __threadfence();
    return S.abort == 0;
}

__device__ void publish(FitGlobal *G)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&G->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Active set (the paper names the heuristic; its definition is in the 2004
// paper).  Candidates: components whose amplitude has the new component's
// sign and whose centre lies inside the new component's window, most recent
// first; skip one closer than max(omega_b, min(s_j, s_m)) to a member already
// taken (the new component first); at most K_max - 1.  FP64 products and sums
// are rounded separately, so membership is reproducible bit for bit.
// ---------------------------------------------------------------------------

__device__ inline bool too_close(double xj, double yj, double sj, double xm, double ym,
                                 double sm, double omega_b)
{
    double ex = __dsub_rn(xj, xm), ey = __dsub_rn(yj, ym);
    double rs = sj < sm ? sj : sm;
    if (rs < omega_b) rs = omega_b;
    return __dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)) <= __dmul_rn(rs, rs);
}

// Start values into S.t0 (thread 0), then the active set, the bounds and the
// published start point.  Whole work-group.
__device__ void setup_fit(const Params &p, FitGlobal *G, WGShared &S, bool use_prop)
{
    const int t = threadIdx.x;
    const double omega_b = p.st->omega_b;
    if (t == 0) {
        const int64_t pr = G->idx / p.W, pc = G->idx % p.W;
        const double pv = G->peak;
        double *t0 = S.t0;
        const double cap = width_cap(p);
        if (use_prop) {
            const double *q = p.st->proposal;
            t0[0] = q[0]; t0[1] = q[1]; t0[2] = q[2]; t0[3] = q[3];
            if (!isfinite(t0[0])) t0[0] = pv;
            if (!(t0[1] >= (double)pc - 16.0)) t0[1] = (double)pc - 16.0;
            if (t0[1] > (double)pc + 16.0) t0[1] = (double)pc + 16.0;
            if (!(t0[2] >= (double)pr - 16.0)) t0[2] = (double)pr - 16.0;
            if (t0[2] > (double)pr + 16.0) t0[2] = (double)pr + 16.0;
            if (t0[1] < 0.0) t0[1] = 0.0;
            if (t0[1] > (double)(p.W - 1)) t0[1] = (double)(p.W - 1);
            if (t0[2] < 0.0) t0[2] = 0.0;
            if (t0[2] > (double)(p.H - 1)) t0[2] = (double)(p.H - 1);
            if (!(t0[3] >= omega_b)) t0[3] = omega_b;
            if (t0[3] > cap) t0[3] = cap;
        } else {
            t0[0] = pv; t0[1] = (double)pc; t0[2] = (double)pr; t0[3] = omega_b;
        }
        make_window(t0[1], t0[2], halfwidth(t0[3], p.window_sigmas), p.H, p.W, S.win[0]);
        S.nch = 0;
        S.sel_done = (p.max_active <= 1) ? 1 : 0;
    }
    __syncthreads();
    const double a0 = S.t0[0], x0 = S.t0[1], y0 = S.t0[2], s0 = S.t0[3];
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
        if (t == 0) {
            for (int w = kT - 1; w >= 0 && !S.sel_done; --w) {
                uint32_t bits = S.mask[w];
                while (bits && !S.sel_done) {
                    const int b = 31 - __clz(bits);
                    bits &= ~(1u << b);
                    const int64_t j = lo + 32 * w + b;
                    const double xj = p.cx[j], yj = p.cy[j], sj = p.cs[j];
                    if (too_close(xj, yj, sj, x0, y0, s0, omega_b)) continue;
                    bool close = false;
                    for (int u = 0; u < S.nch && !close; ++u) {
                        const int64_t mj = S.members[u + 1];
                        close = too_close(xj, yj, sj, p.cx[mj], p.cy[mj], p.cs[mj], omega_b);
                    }
                    if (close) continue;
                    S.members[1 + S.nch] = (int32_t)j;
                    S.nch++;
                    if (S.nch >= p.max_active - 1) S.sel_done = 1;
                }
            }
        }
    }
    __syncthreads();
    const int m = 1 + S.nch;
    if (t == 0) {
        S.members[0] = -1;
        G->m = m;
        G->n = 4 * m;
        G->phase = 0;
        G->trials = 0;
        G->converged = 0;
    }
    __syncthreads();
    if (t < m) {
        double th[4];
        if (t == 0) {
            th[0] = a0; th[1] = x0; th[2] = y0; th[3] = s0;
        } else {
            const int64_t j = S.members[t];
            th[0] = p.ca[j]; th[1] = p.cx[j]; th[2] = p.cy[j]; th[3] = p.cs[j];
        }
        int32_t w[4];
        make_window(th[1], th[2], halfwidth(th[3], p.window_sigmas), p.H, p.W, w);
        // bounds: the start sign of the amplitude; the centre inside its start
        // window; omega_b <= s <= the width cap
        const bool neg = th[0] < 0.0;
        const double lo4[4] = {neg ? -INFINITY : 0.0, (double)w[2], (double)w[0], omega_b};
        const double hi4[4] = {neg ? 0.0 : INFINITY, (double)w[3], (double)w[1], width_cap(p)};
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * t + q;
            G->lo[i] = lo4[q];
            G->hi[i] = hi4[q];
            G->th0[i] = th[q];
            G->th_old[i] = (t == 0) ? 0.0 : th[q];
            double v = th[q];
            if (!(v >= lo4[q])) v = lo4[q];
            if (v > hi4[q]) v = hi4[q];
            G->th_e[i] = v;
        }
        G->members[t] = S.members[t];
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

// Member constants at theta = G->th_e and the old members' stored Gaussians.
__device__ void prepare(const Params &p, FitGlobal *G, WGShared &S)
{
    const int t = threadIdx.x;
    if (t == 0) { S.m = G->m; S.n = G->n; }
    __syncthreads();
    if (t < S.m) {
        const double a = G->th_e[4 * t], x = G->th_e[4 * t + 1], y = G->th_e[4 * t + 2],
                     s = G->th_e[4 * t + 3];
        make_window(x, y, halfwidth(s, p.window_sigmas), p.H, p.W, S.win[t]);
        const double s2 = s * s;
        S.mx[t] = x;
        S.my[t] = y;
        S.mamp[t] = a;
        S.minv2[t] = 1.0 / (2.0 * s2);
        S.minvs2[t] = 1.0 / s2;
        S.minvs3[t] = 1.0 / (s2 * s);
        if (t > 0) {
            const double oa = G->th_old[4 * t], ox = G->th_old[4 * t + 1],
                         oy = G->th_old[4 * t + 2], os = G->th_old[4 * t + 3];
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

// Tiles tile0, tile0 + stride, ... of U; the work-group's partial (FP64:
// n_out Gram entries, F, chi2, the pixel count) goes to out.
__device__ void evaluate_tiles(const Params &p, WGShared &S, float *tile, double *red,
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
    int64_t npx = 0;
    double f_acc = 0.0, c_acc = 0.0;
    float *row = tile + t * kTileStride;
    for (int64_t ti = tile0; ti < ntiles; ti += stride) {
        const int64_t lin = ti * kT + t;
        bool valid = false;
        int32_t r = 0, c = 0;
        if (lin < total) {
            int w = 0;
            while (lin >= S.pref[w + 1]) ++w;
            const int64_t local = lin - S.pref[w];
            const int32_t wc = S.win[w][3] - S.win[w][2] + 1;
            r = S.win[w][0] + (int32_t)(local / wc);
            c = S.win[w][2] + (int32_t)(local % wc);
            valid = true;
            for (int i = 0; i < w; ++i)
                if (in_box(S.win[i], r, c)) { valid = false; break; }
        }
        if (valid) {
            ++npx;
            double D = (double)p.R[(int64_t)r * p.W + c];
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
#pragma unroll
        for (int u = 0; u < kOwnMax; ++u) {
            if (u >= n_own) break;
            const int ci = oi[u], ck = ok_[u];
            float sum = acc_s[u], comp = acc_c[u];
            for (int q = my_s; q < kT; q += S_sub) {
                const float *rq = tile + q * kTileStride;
                const float y = rq[ci] * rq[ck] - comp;
                const float tt = sum + y;
                comp = (tt - sum) - y;
                sum = tt;
            }
            acc_s[u] = sum;
            acc_c[u] = comp;
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
    // F, chi2 and the pixel count, summed over the threads in a fixed order
    const double vals[3] = {f_acc, c_acc, (double)npx};
    for (int q = 0; q < 3; ++q) {
        __syncthreads();
        red[t] = vals[q];
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int i = 0; i < kT; ++i) s += red[i];
            out[n_out + q] = s;
        }
    }
    __syncthreads();
}

// Sum the partials of work-groups 0..geff-1 in that order into He, S.ge,
// S.Fe, S.chi2e, S.npx_e.
__device__ void reduce_partials(const Params &p, WGShared &S, int geff, double *He)
{
    const int t = threadIdx.x;
    const int n = S.n;
    const int n_out = (n + 1) * (n + 2) / 2;
    for (int o = t; o < n_out + 3; o += kT) {
        double v = 0.0;
        for (int w = 0; w < geff; ++w) v += p.partials[(int64_t)w * kPartStride + o];
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

// Work-group Cholesky solve of A x = b (A n x n in LDS, overwritten).
__device__ bool chol_solve(WGShared &S, double *A, int n, double *b, double *x)
{
    const int t = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        if (t == 0) {
            const double d = A[k * n + k];
            S.ok = (d > 0.0 && isfinite(d)) ? 1 : 0;
            if (S.ok) A[k * n + k] = sqrt(d);
        }
        __syncthreads();
        if (!S.ok) return false;
        for (int i = k + 1 + t; i < n; i += kT) A[i * n + k] /= A[k * n + k];
        __syncthreads();
        const int rem = n - k - 1;
        for (int e = t; e < rem * rem; e += kT) {
            const int i = k + 1 + e / rem, j = k + 1 + e % rem;
            if (j <= i) A[i * n + j] -= A[i * n + k] * A[j * n + k];
        }
        __syncthreads();
    }
    for (int i = 0; i < n; ++i) {
        if (t == 0) x[i] = b[i] / A[i * n + i];
        __syncthreads();
        for (int j = i + 1 + t; j < n; j += kT) b[j] -= A[j * n + i] * x[i];
        __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {
        if (t == 0) x[i] = x[i] / A[i * n + i];
        __syncthreads();
        for (int j = t; j < i; j += kT) x[j] -= A[i * n + j] * x[i];
        __syncthreads();
    }
    if (t == 0) {
        int good = 1;
        for (int i = 0; i < n; ++i) good &= isfinite(x[i]) ? 1 : 0;
        S.ok = good;
    }
    __syncthreads();
    return S.ok != 0;
}

// ---------------------------------------------------------------------------
// The LM bookkeeping (Marquardt 1963) after one evaluation, by the reducing
// work-group.  Damped system (H + mu D) delta = g with
// D = diag(max(H_ii, 1e-12 max H_ii)); a parameter on a bound whose gradient
// leaves the box is held for the trial; the trial point is clipped to the
// bounds; accept iff F decreases; gain-ratio damping (mu *= max(1/3,
// 1 - (2 rho - 1)^3) on accept, mu *= nu, nu *= 2 on reject); converged when
// an accepted step has max |delta_k| / scale_k < tol, or stalled once mu
// passes 1e8; the budget counts trials.
// Sets S.finished when the fit is over; otherwise G->th_e holds the next
// trial.
// ---------------------------------------------------------------------------

__device__ void lm_step(const Params &p, FitGlobal *G, WGShared &S, double *He, double *A)
{
    const int t = threadIdx.x;
    const int n = S.n, m = S.m;
    if (t == 0) {
        S.finished = 0;
        if (G->phase == 0) {
            S.accept = 1;
            G->mu = p.lm_mu0;
            G->nu = 2.0;
            G->trials = 0;
            G->converged = 0;
            G->chi2_init = S.chi2e;
            G->phase = 1;
        } else {
            double Ft = S.Fe;
            if (!isfinite(Ft)) Ft = INFINITY;
            S.accept = (Ft < G->F_c) ? 1 : 0;
            if (S.accept) {
                double step = 0.0;
                for (int j = 0; j < m; ++j) {
                    const double *tn = G->th_e + 4 * j, *to = G->th_c + 4 * j;
                    const double sa = fabs(tn[0]) > 1e-30 ? fabs(tn[0]) : 1e-30;
                    double v;
                    v = fabs(tn[0] - to[0]) / sa; step = v > step ? v : step;
                    v = fabs(tn[1] - to[1]) / tn[3]; step = v > step ? v : step;
                    v = fabs(tn[2] - to[2]) / tn[3]; step = v > step ? v : step;
                    v = fabs(tn[3] - to[3]) / tn[3]; step = v > step ? v : step;
                }
                const double rho = G->pred > 0.0 ? (G->F_c - Ft) / G->pred : 1.0;
                const double tt = 2.0 * rho - 1.0;
                double f = 1.0 - tt * tt * tt;
                if (f < 1.0 / 3.0) f = 1.0 / 3.0;
                G->mu *= f;
                if (G->mu < 1e-12) G->mu = 1e-12;
                G->nu = 2.0;
                if (step < p.lm_tol) { G->converged = 1; S.finished = 1; }
            } else {
                G->mu *= G->nu;
                G->nu *= 2.0;
                if (G->mu > 1e8) { G->converged = 1; S.finished = 1; }
            }
        }
    }
    __syncthreads();
    if (S.accept) {
        for (int e = t; e < n * n; e += kT) G->Hc[e] = He[e];
        if (t < n) { G->th_c[t] = G->th_e[t]; G->g_c[t] = S.ge[t]; }
        if (t == 0) { G->F_c = S.Fe; G->chi2_c = S.chi2e; G->npx_c = S.npx_e; }
        // the reducer reads Hc back below: its own writes, ordered by the barrier
        __threadfence_block();
    }
    __syncthreads();
    // next trial point, or finished
    for (;;) {
        __syncthreads();
        if (S.finished) break;
        if (t == 0) {
            if (G->trials >= p.lm_max_iter) {
                S.finished = 1;
            } else {
                double dmax = 0.0;
                for (int i = 0; i < n; ++i) dmax = G->Hc[i * n + i] > dmax ? G->Hc[i * n + i] : dmax;
                for (int i = 0; i < n; ++i) {
                    const double d = G->Hc[i * n + i];
                    S.dd[i] = d < 1e-12 * dmax ? 1e-12 * dmax : d;
                    const double th = G->th_c[i], g = G->g_c[i];
                    S.frozen[i] = ((th <= G->lo[i] && g <= 0.0) || (th >= G->hi[i] && g >= 0.0)) ? 1 : 0;
                    S.rhs[i] = S.frozen[i] ? 0.0 : g;
                }
                G->trials++;
            }
        }
        __syncthreads();
        if (S.finished) break;
        const double mu = G->mu;
        for (int e = t; e < n * n; e += kT) {
            const int i = e / n, k = e % n;
            double v;
            if (S.frozen[i] || S.frozen[k]) v = (i == k) ? 1.0 : 0.0;
            else v = G->Hc[e] + (i == k ? mu * S.dd[i] : 0.0);
            A[e] = v;
        }
        if (t < n) S.rhs_copy[t] = S.rhs[t];
        __syncthreads();
        const bool ok = chol_solve(S, A, n, S.rhs_copy, S.delta);
        if (ok) {
            if (t == 0) {
                double pred = 0.0;
                for (int i = 0; i < n; ++i) {
                    double v = G->th_c[i] + S.delta[i];
                    pred += S.delta[i] * (S.rhs[i] + mu * S.dd[i] * S.delta[i]);
                    if (!(v >= G->lo[i])) v = G->lo[i];
                    if (v > G->hi[i]) v = G->hi[i];
                    G->th_e[i] = v;
                }
                G->pred = pred;
            }
            __syncthreads();
            break;
        }
        if (t == 0) {       // not positive definite: treated as a rejected trial
            G->mu *= G->nu;
            G->nu *= 2.0;
            if (G->mu > 1e8) { G->converged = 1; S.finished = 1; }
        }
    }
    __syncthreads();
}

// Commit (Sect. 3: the loop gain on the new component; refits replace the
// old members) and the residual-update plan.  Whole work-group.
__device__ void commit(const Params &p, FitGlobal *G, WGShared &S)
{
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int m = S.m;
    if (t == 0) {
        const int64_t L = st->L, k = st->k;
        st->n_active = m;
        st->lm_iters = G->trials_total + G->trials;
        st->converged = G->converged;
        st->used_fallback = G->used_fallback;
        st->chi2_init = G->chi2_init;
        st->chi2_final = G->chi2_c;
        st->fit_px = G->npx_c;
        st->sum_trials += (unsigned long long)(G->trials_total + G->trials);
        st->not_converged += G->converged ? 0ull : 1ull;
        st->fallbacks += (unsigned long long)G->used_fallback;
        st->have_proposal = 0;
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
            const int64_t cj = G->members[j];
            const double *to = G->th_old + 4 * j, *tn = G->th_c + 4 * j;
            add_rect(to[0], to[1], to[2], to[3], +1.0f);
            add_rect(tn[0], tn[1], tn[2], tn[3], -1.0f);
            p.ca[cj] = tn[0]; p.cx[cj] = tn[1]; p.cy[cj] = tn[2]; p.cs[cj] = tn[3];
            p.c_updated[cj] = k;
        }
        const double anew = p.gain * G->th_c[0];
        add_rect(anew, G->th_c[1], G->th_c[2], G->th_c[3], -1.0f);
        p.ca[L] = anew; p.cx[L] = G->th_c[1]; p.cy[L] = G->th_c[2]; p.cs[L] = G->th_c[3];
        p.c_added[L] = k;
        p.c_updated[L] = k;
        st->n_rects = nr;
        st->bb[0] = bb[0]; st->bb[1] = bb[1]; st->bb[2] = bb[2]; st->bb[3] = bb[3];
        st->update_px = 0ull;
        st->L = L + 1;
        st->k = k + 1;
        st->fit_ready = 1;
    }
    if (t < m) st->members[t] = G->members[t];
    if (t < 4 * m) {
        st->theta0[t] = G->th0[t];
        st->theta[t] = G->th_c[t];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kT) void k_fit(Params p)
{
    extern __shared__ __align__(16) unsigned char lds[];
    float *tile = reinterpret_cast<float *>(lds);
    double *A = reinterpret_cast<double *>(tile + kT * kTileStride);
    double *He = A + kMaxN * kMaxN;
    double *red = He + kMaxN * kMaxN;
    __shared__ WGShared S;
    FitGlobal *G = p.fg;
    DevState *st = p.st;
    const int t = threadIdx.x;
    const int wg = blockIdx.x, nwg = gridDim.x;

    // Nothing writes the stop flag before every work-group has checked in, so
    // all of them agree here.
    if (st->stop) return;

    // Check in: every work-group reads the generation before work-group 0 may
    // publish.
    if (t == 0) {
        S.gen = __hip_atomic_load(&G->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        S.abort = 0;
        __hip_atomic_fetch_add(&G->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (wg == 0) {
        if (t == 0) {
            long it = 0;
            while (__hip_atomic_load(&G->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                       (unsigned)nwg && it < kSpinLimit) {
                __builtin_amdgcn_s_sleep(2);
                ++it;
            }
            S.abort = it >= kSpinLimit ? 1 : 0;
            __threadfence();
            __hip_atomic_store(&G->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the peak and the stop test (Sect. 2 steps 1 and 4)
            st->fit_ready = 0;
            const unsigned long long key = st->peak_key;
            st->peak_key = 0ull;
            int64_t idx = st->forced_idx >= 0
                              ? st->forced_idx
                              : (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
            const bool bad_idx = (st->forced_idx < 0 && key == 0ull) || idx < 0 || idx >= p.H * p.W;
            st->forced_idx = -1;
            S.stop = 0;
            if (S.abort) S.stop = ASP_ERR_DEVICE;
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
            G->idx = idx;
            G->peak = (double)v;
            G->pass = 0;
            G->trials_total = 0;
            G->used_fallback = 0;
            G->use_prop = (p.use_proposal && st->have_proposal) ? 1 : 0;
            G->done = S.stop ? 1 : 0;
            if (S.stop) st->stop = S.stop;
        }
        __syncthreads();
        if (!S.stop) setup_fit(p, G, S, G->use_prop != 0);
        publish(G);
    }
    for (;;) {
        if (!wait_publish(G, S)) {
            if (t == 0) st->stop = ASP_ERR_DEVICE;
            return;
        }
        if (t == 0) S.done = G->done;
        __syncthreads();
        if (S.done) return;
        prepare(p, G, S);
        const int64_t ntiles = (S.pref[S.m] + kT - 1) / kT;
        const int geff = (int)(ntiles < nwg ? ntiles : nwg);
        if (wg >= geff) continue;
        evaluate_tiles(p, S, tile, red, wg, geff, p.partials + (int64_t)wg * kPartStride);
        __threadfence();
        __syncthreads();
        if (t == 0) {
            const unsigned prev =
                __hip_atomic_fetch_add(&G->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            S.last = (prev == (unsigned)geff - 1u) ? 1 : 0;
        }
        __syncthreads();
        if (!S.last) continue;
        // The reducing work-group.
        if (t == 0) __hip_atomic_store(&G->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __syncthreads();
        reduce_partials(p, S, geff, He);
        lm_step(p, G, S, He, A);
        if (S.finished) {
            if (G->use_prop && !G->converged && G->pass == 0) {
                // the learned start did not converge: the simple values instead
                if (t == 0) {
                    G->trials_total += G->trials;
                    G->used_fallback = 1;
                    G->pass = 1;
                }
                __syncthreads();
                setup_fit(p, G, S, false);
            } else {
                commit(p, G, S);
                if (t == 0) G->done = 1;
            }
        }
        publish(G);
    }
}

hipError_t fit_kernel_setup()
{
    return hipFuncSetAttribute((const void *)k_fit, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kFitLds);
}

int fit_grid_size(int device)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fit, kT, kFitLds) !=
            hipSuccess || per_cu < 1)
        return 1;
    const int g = cus * per_cu;
    return g < 1 ? 1 : g;
}

hipError_t launch_fit(const Params &p, hipStream_t s)
{
    void *args[] = {(void *)&p};
    return hipLaunchCooperativeKernel((const void *)k_fit, dim3(p.fit_grid), dim3(kT), args,
                                      kFitLds, s);
}

}  // namespace asp
