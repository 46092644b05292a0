// Internal declarations of the gfx950 minor cycle: device state, launch
// parameters, geometry helpers and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asp.h"

namespace asp {

constexpr int kMaxM = ASP_MAX_ACTIVE;          // members of one fit
constexpr int kMaxN = 4 * kMaxM;               // parameters of one fit
constexpr int kMaxRects = 2 * (kMaxM - 1) + 1; // windows touched by one update
constexpr int kFitThreads = 256;               // work-group of the fit kernel
constexpr int kCols = kMaxN + 1;               // J columns + residual
constexpr int kTileStride = kCols + 1;         // padded LDS row

// A signed Gaussian on a window, one term of the residual update.
struct Rect {
    int32_t r0, r1, c0, c1;
    double a, x, y, s;
    float sign;
    int32_t pad;
};

constexpr int kProfSlots = 14;

constexpr int kPeakSlots = 64;   // wave-size: one slot per lane of the collecting wave

// The incremental peak search: the packed peak key of every kPkTile x kPkTile
// tile of R, and the list of tiles that residual updates touched since the
// last search.  tiles_x = 0: the peak search scans the whole image.  It lives
// in the device state, not in the launch parameters.
constexpr int kPkTile = 64;
struct PeakTiles {
    unsigned long long *keys;      // per tile: (|v| bits << 32) | (0xFFFFFFFF - idx)
    int32_t *dirty, *list;         // per tile: stale flag; the stale tiles, each once
    unsigned int *count;           // entries in list
    int32_t tiles_x, tiles_y;
};


// Mutable per-context state in device memory.
struct DevState {
    // packed keys (|v| bits << 32) | (0xFFFFFFFF - idx), one slot per
    // work-group index mod kPeakSlots; the peak is their maximum
    unsigned long long peak_keys[kPeakSlots];
    int32_t stop;                  // 0 running, ASP_STOP_*, or ASP_ERR_CAPACITY
    int32_t fit_ready;             // 1 between a fit and its residual update
    int64_t k;                     // iterations done
    int64_t L;                     // components
    int64_t forced_idx;            // >= 0: fit this pixel instead of the peak key
    int64_t idx;                   // pixel of the last fit
    float peak;                    // residual there before the fit
    int32_t have_proposal;         // 1 caller's proposal, 2 the network's, 0 none
    double proposal[4];            // convolved-space (a, x, y, s), before clamping
    // report of the last fit
    int32_t n_active, lm_iters, converged, used_fallback;
    int32_t members[kMaxM];
    int32_t init_source;           // have_proposal of the last fit
    int32_t start_prop;            // its LM started from the proposal
    double init[4];                // its proposal
    double chi2_init, chi2_final;
    double theta0[kMaxN], theta[kMaxN];
    int64_t fit_px;
    int32_t added;                 // the new component joined the list
    int32_t pad_a;
    // update plan
    int32_t n_rects, pad0;
    Rect rects[kMaxRects];
    int32_t bb[4];                 // bounding box of the rects
    // counters summed over iterations
    unsigned long long sum_trials, not_converged, fallbacks;
    unsigned long long not_added;       // fits whose new component had amplitude zero
    unsigned long long px_total;        // pixels read-modify-written by the updates so far
                                        // (written by k_px_read from px_slots)
    unsigned long long sum_eval_px;     // pixel evaluations of the LM trials
    unsigned long long sum_gram_flops;  // (n+1)(n+2) per pixel evaluation
    // Gaussian main lobe of the PSF
    double alpha_b, omega_b;
    int64_t lobe_px;
    int32_t psf_status, pad1;
    // fit phase timers (device wall clock ticks) and event counts
    unsigned long long prof[kProfSlots];
    // per active-set size m: fits, their LM trials and their wall-clock ticks
    // (start values to commit)
    unsigned long long fits_m[kMaxM + 1], trials_m[kMaxM + 1], ticks_m[kMaxM + 1];
    // training-sample recording: slots filled
    int64_t rec_n;
    // the smoothing method: this iteration smooths; smooth_start is current
    int32_t smooth_now, smooth_ready;
    int32_t smooth_scale, pad2;    // scale j of the start
    int64_t smooth_idx;            // its pixel
    float smooth_score, pad3;      // its |score| as compared
    double smooth_start[4];        // (a, x, y, s)
    unsigned long long sum_smoothed;    // fits started from it
    unsigned long long sm_px[2 * ASP_MAX_SCALES];  // image pixels through the column
                                                   // (j) and row (8 + j) passes
    unsigned long long pk_tiles_done;   // tiles rescanned by the incremental peak search
    PeakTiles pk;                       // the incremental peak search's buffers
    // the tracked sum of R^2: sq_base (a full pass at the last wholesale change
    // of R) plus the windowed deltas of the updates since, one slot per update
    // work-group index
    double *sq_slots;
    int32_t sq_nslots, sq_pad;
    double sq_base;
    // pixels rewritten by the updates, one running count per update
    // work-group index (no two work-groups add to one counter)
    unsigned long long *px_slots;
    // one evaluation of a given trial (asp_eval_trial): diag_m > 0 members,
    // their parameters and the old members' stored ones; the reduced sums go
    // to diag_out: J^T J (n x n), J^T r (n), F, chi2, the pixel count
    int32_t diag_m, pad_d;
    double diag_theta[kMaxN], diag_stored[kMaxN];
    double *diag_out;
};
constexpr int kSqSlots = 4096;

// State of one fit shared by the work-groups of the fit kernel.  The
// published part (m .. th_old) is written by one work-group and read by all
// after the generation counter moves; the LM part is touched only by the
// work-group that reduces a trial.
constexpr int kNOutMax = (kMaxN + 1) * (kMaxN + 2) / 2;       // augmented Gram entries
constexpr int kPartStride = kNOutMax + 3;                      // + F, chi2 (FP64), pixels
constexpr int kMaxGroups = 64;     // partial rows beyond the grid, one per arrival group

struct FitGlobal {
    int32_t m, n, done, cmd;            // cmd, field: the batched kernel's command
    int32_t field, pad0;
    double th_e[kMaxN];                 // parameters under evaluation
    double th_old[kMaxN];               // stored parameters of the old members
    unsigned int gen;                   // publication counter
    unsigned int beat;                  // the batched leader's iteration heartbeat
    unsigned int top;                   // second-level arrivals (one per group)
    unsigned int arrive_g[kMaxGroups];  // first-level arrivals (one per work-group)
};

// The smoothing method's kernels: trial widths, taps and the device copy of
// the smoothed images.  Output tiles are kSmTile x kSmTile pixels; a thread
// computes kSmRb consecutive outputs along the filter axis.
constexpr int kMaxScales = ASP_MAX_SCALES;
constexpr int kSmTile = 64;
constexpr int kSmRb = 16;
struct SmoothParams {
    float *vt;                     // n planes W x H: the column pass, transposed
    const float *taps;             // scale j at off[j]: kSmRb nb[j] taps, zero past 2h
    const float *wx, *wy;          // scale j at j W (j H): 1 / sqrt(row sum of k^2) (norm 1)
    unsigned long long *keys;      // n x ntiles: per tile and scale, the packed maximum
    int32_t *dirty_a, *dirty_b;    // n x ntiles: tile of the column (row) pass is stale
    int32_t *list_a, *list_b;      // the stale entries j ntiles + tile, each once
    unsigned int *count;           // entries in list_a, list_b
    float *map;                    // optional H x W output of one scale's smoothed image
    int32_t map_scale;
    int32_t n, norm, switch_area;
    int32_t tiles_x, tiles_y;
    int32_t h[kMaxScales], nb[kMaxScales], off[kMaxScales];
    double sig[kMaxScales];
};

// Read-only launch parameters.
struct Params {
    float *R;                      // residual H x W
    int64_t H, W;
    double *ca, *cx, *cy, *cs;     // component list (SoA, FP64)
    int64_t *c_added, *c_updated;
    int64_t cap;
    DevState *st;
    double gain, threshold;
    int64_t max_iter;
    int32_t max_active, lm_max_iter;
    double window_sigmas, max_width, lm_mu0, lm_tol;
    int32_t use_proposal;          // honour st->proposal when have_proposal
    int32_t fit_grid;              // work-groups of the fit kernel
    int32_t solo_tiles;            // trials of at most this many tiles: work-group 0 alone
    int32_t min_tiles;             // least tiles per work-group in a shared trial
    unsigned long long spin_ticks; // time bound of every wait between work-groups
    int32_t group;                 // work-groups per first-level arrival counter
    int32_t fuse_update;           // k_fit ends with the residual update on all its work-groups
    FitGlobal *fg;
    double *partials;              // fit_grid x kPartStride
    // recording of (patch, target) training pairs; rec_cap = 0 disables
    float *rec_patch;              // rec_cap x 1024
    float *rec_target;             // rec_cap x 4
    int32_t *rec_flag;             // rec_cap: 1 converged fit from the simple values
    int64_t rec_cap;
    int32_t smooth;                // the smoothing method and its switch are on
    int32_t pad_s;
    SmoothParams sm;
};

// The proposal network in the layout of the inference kernel: W1 row-major
// (as trained), W2 transposed (input-major), then W3 and the biases.  The
// kernel runs kPropGroups work-groups, each owning kNetH / kPropGroups units
// of the first hidden layer; their partial sums of the second layer and an
// arrival counter sit in a scratch area of kNetScratch floats after the
// weights.
constexpr int kNetIn = 1024, kNetH = 256, kNetOut = 4, kPatch = 32, kPatchHalf = 16;
constexpr int64_t kNetParams = (int64_t)kNetH * kNetIn + kNetH + (int64_t)kNetH * kNetH + kNetH +
                               (int64_t)kNetOut * kNetH + kNetOut;
constexpr int kPropGroups = 64;
constexpr int64_t kNetScratch = (int64_t)kPropGroups * kNetH + 64;
struct NetParams {
    const float *w1, *b1, *w2t, *b2, *w3, *b3;
    float *part;                   // kPropGroups x kNetH second-layer partial sums
    unsigned int *done;            // arrivals, counted modulo kPropGroups
};

// ---------------------------------------------------------------------------
// Geometry (window rule of the fit and the update).  FP64 products and sums
// are written so that no two roundings fuse into one.
// ---------------------------------------------------------------------------

__host__ __device__ inline int halfwidth(double s, double window_sigmas)
{
    double h = ceil(window_sigmas * s);
    if (!(h >= 3.0)) h = 3.0;
    if (h > 1073741823.0) h = 1073741823.0;
    return (int)h;
}

// Window of half-width h around (floor(x + 0.5), floor(y + 0.5)), clipped.
__host__ __device__ inline void make_window(double x, double y, int h, int64_t H, int64_t W,
                                            int32_t box[4])
{
    int64_t cx = (int64_t)floor(x + 0.5), cy = (int64_t)floor(y + 0.5);
    int64_t r0 = cy - h, r1 = cy + h, c0 = cx - h, c1 = cx + h;
    box[0] = (int32_t)(r0 < 0 ? 0 : r0);
    box[1] = (int32_t)(r1 > H - 1 ? H - 1 : r1);
    box[2] = (int32_t)(c0 < 0 ? 0 : c0);
    box[3] = (int32_t)(c1 > W - 1 ? W - 1 : c1);
}

__host__ __device__ inline bool in_box(const int32_t b[4], int32_t r, int32_t c)
{
    return r >= b[0] && r <= b[1] && c >= b[2] && c <= b[3];
}

__device__ inline double width_cap(const Params &p)
{
    double m = p.max_width > 0.0 ? p.max_width
                                 : (double)(p.H < p.W ? p.H : p.W) / 8.0;
    return m > p.st->omega_b ? m : p.st->omega_b;
}

// The peak key: the maximum over the slots, read by the 64 lanes of wave 0
// (lanes of other waves get 0).  With reset, the slots are cleared after the
// read.  Every thread of the work-group must call it.
__device__ inline unsigned long long collect_peak_key(DevState *st, bool reset,
                                                      unsigned long long *lds_key)
{
    const int t = threadIdx.x;
    if (t < 64) {
        // atomic accesses: the slots are written by atomics at L2, possibly by
        // this work-group moments before
        unsigned long long k = __hip_atomic_load(&st->peak_keys[t], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        if (reset)
            __hip_atomic_store(&st->peak_keys[t], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(k, off, 64);
            k = o > k ? o : k;
        }
        if (t == 0) *lds_key = k;
    }
    __syncthreads();
    return *lds_key;
}

// Launchers (kernels.hip).
hipError_t launch_peak(const Params &p, int grid, hipStream_t s);
hipError_t launch_peak_decode(const Params &p, hipStream_t s);
hipError_t launch_fit(const Params &p, hipStream_t s);
hipError_t launch_update(const Params &p, int grid, hipStream_t s);
hipError_t launch_psf_fit(const float *psf, int64_t Hp, int64_t Wp, double lobe_frac,
                          DevState *st, int32_t *work, hipStream_t s);
hipError_t launch_check_finite(const float *img, int64_t n, int32_t *flag, hipStream_t s);
hipError_t launch_components(const Params &p, asp_component *out, hipStream_t s);
// The smoothing method: refresh of the stale tiles of the smoothed images
// (both passes) and the pick of the peak.  force = 0: only when the device
// state says this iteration smooths; 1: always; 2: always, and every tile of
// the row pass is recomputed (the column pass keeps to its stale tiles).
hipError_t launch_smooth_passes(const Params &p, int force, hipStream_t s);
hipError_t launch_smooth_pick(const Params &p, int force, hipStream_t s);
// Every tile of every scale stale, both passes.
hipError_t launch_smooth_mark_all(const Params &p, hipStream_t s);
// The exact-PSF residual refresh: its own argument block (the launch
// parameters of the minor cycle stay within 512 bytes).  grid: Py x Px FP64,
// the zero-padded model and then the convolution; spec / pspec: Py x
// (Px / 2 + 1) complex spectra of the model and of the PSF.
struct RefreshArgs {
    const float *dirty, *psf;
    float *R;
    const double *ca, *cx, *cy, *cs;
    DevState *st;
    double *grid;
    double2 *spec;
    double2 *pspec;
    int64_t H, W, Hp, Wp, Py, Px;
    int32_t ci, cj;                // the PSF's peak pixel
    double window_sigmas;
    int32_t force;                 // 1: also when the stop flag is set
    int32_t pad;
};
hipError_t refresh_psf_spectrum(const RefreshArgs &a, void *plan_fwd, hipStream_t s);
hipError_t refresh_residual(const RefreshArgs &a, void *plan_fwd, void *plan_inv, hipStream_t s);
// The model image (the refresh's rendering, no convolution) into out, H x W FP32.
hipError_t render_model(const RefreshArgs &a, float *out, hipStream_t s);

// The Asp-Clean2004 iteration (Sect. 2 steps 1-4 with the objective of
// Eq. 3): Levenberg-Marquardt state of the one sky component (F, x, y,
// omega^2) being fitted, kept on the device between the evaluations.
struct A4State {
    double theta[4];               // accepted point
    double te[4];                  // point under evaluation
    double theta0[4];              // start after the bounds
    double lo[4], hi[4];
    double Hs[16], g[4];           // J^T J and J^T r at theta
    double dd[4];                  // the damping's diagonal of the last trial
    double F, chi2, F0, chi2_init; // F = sum m (m - 2 R); chi2 = sum (R - m)^2
    double mu, nu, pred;
    int32_t trials, converged, done, phase;   // phase 0: the start is evaluated next
    int32_t evals, pad;
};
constexpr int kA4Sums = 16;        // 10 Gram entries, 4 of J^T r, F, chi2
constexpr int kA4Blocks = 1024;    // partial rows of an evaluation
constexpr int kA4RowBlocks = 2048; // work-groups of the direct convolution's row pass

struct A4Args {
    float *R;
    DevState *st;
    A4State *s;
    double *ca, *cx, *cy, *cs;
    int64_t *c_added, *c_updated;
    int64_t cap;
    double *grid;                  // 4 images Py x Px: B(*) of g, dg/dx, dg/dy, dg/d(omega^2)
    double2 *spec;                 // their half spectra, Py x (Px/2 + 1) each
    double2 *fac;                  // 1-D DFTs of the factors: 3 Py rows, then 3 (Px/2 + 1)
    const double2 *pspec;          // the PSF's
    double *partials;              // nblk x kA4Sums
    const float *psf;              // the PSF, Hp x Wp (direct convolution)
    double *taps;                  // per-axis factors: 3 W column taps, then 3 H row taps
    int32_t *tapi;                 // C0, nc, R0, nr of the factors
    int64_t grid_cap;              // doubles in grid (4 Py Px)
    int64_t Hp, Wp;
    int64_t H, W, Py, Px;
    int32_t ci, cj;                // the PSF's peak pixel
    int32_t budget;
    int32_t nblk;                  // work-groups of the sums: min(kA4Blocks, H)
    double gain, window_sigmas, s_max, mu0, tol;
};
// Stop test after the peak, the start from the smoothing method, bounds.
hipError_t a4_begin(const A4Args &a, hipStream_t s);
// One evaluation of Eq. 3 and its Jacobian at s->te, then the LM decision and
// the next trial point (or done).  plan_inv4: the batched (4) Z2D.
hipError_t a4_trial(const A4Args &a, void *plan_inv4, hipStream_t s);
// The residual update R -= gain B (*) g(theta) and the new component
// (plan_inv: the single Z2D).
hipError_t a4_commit(const A4Args &a, void *plan_inv, hipStream_t s);
// The same two steps with B (*) g formed directly: a pass along the rows of the
// PSF with the column factors into the grids (3 planes of (H + nr - 1) x W for
// an evaluation, 1 for the update; the caller checks that they fit), then a
// pass along the columns with the row factors.
hipError_t a4_trial_direct(const A4Args &a, hipStream_t s);
hipError_t a4_commit_direct(const A4Args &a, hipStream_t s);

// The incremental peak search: rescan the stale tiles, then reduce the tile
// keys into the peak key; and every tile stale.
hipError_t launch_peak_tiles(const Params &p, int ntiles, hipStream_t s);
hipError_t launch_peak_mark_all(const Params &p, hipStream_t s);
hipError_t launch_propose(const Params &p, const NetParams &net, int use_net, hipStream_t s);
// The tracked sum of R^2: re-based on a full pass (*total) with the slots
// cleared, and read (base plus the slots in a fixed order) into *out.
hipError_t launch_sq_rebase(DevState *st, const double *total, hipStream_t s);
hipError_t launch_sq_read(DevState *st, double *out, hipStream_t s);
// st->px_total = the sum of st->px_slots.
hipError_t launch_px_read(DevState *st, hipStream_t s);
hipError_t launch_sumsq(const float *img, int64_t n, double *part, int nblk, double *out,
                        hipStream_t s);
hipError_t fit_kernel_setup();
// Work-groups of the cooperative fit launch: every one resident at once (the
// occupancy at the kernel's LDS times the CUs) -- 0 when the kernel needs a
// private segment (scratch), with which the waves of one launch are not
// guaranteed to be resident together.
int fit_grid_size(int device);

// The batched kernel: many fields, one persistent launch (fit.hip).
struct BatchArgs {
    const Params *fields;          // n_fields parameter blocks (device)
    const int32_t *order;          // fields in the order teams take them
    unsigned int *queue;           // next position in order (reset before each launch)
    FitGlobal *fg;                 // one per team
    double *partials;              // per team (T + groups) x kPartStride
    int64_t n_iter;                // iterations per field in this launch
    int64_t solo_peak_px;          // peak search by the leader alone up to this many pixels
    int64_t solo_update_px;        // update by the leader alone up to this bounding box
    unsigned long long spin_ticks; // time bound of every wait between work-groups
    int32_t n_fields, team_size, solo_tiles, min_tiles;
};
// Work-groups of the persistent batched launch, whole XCD rows that are all
// resident at once; 0 when that cannot be guaranteed (a private segment, or
// no occupancy).
int batch_grid_size(int device);
hipError_t launch_batch(const BatchArgs &b, int grid, hipStream_t s);

}  // namespace asp
