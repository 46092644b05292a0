// Host runtime of the C ABI declared in include/asp.h: context lifetime,
// argument checks, the step API and the device-resident run loop.  No C++
// exception crosses the ABI; every HIP failure becomes ASP_ERR_DEVICE with a
// message kept in the context.
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include <hipfft/hipfft.h>

#include "asp_device.h"

using asp::DevState;
using asp::Params;

struct asp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t H = 0, W = 0, Hp = 0, Wp = 0;
    asp_options opt{};
    float *R = nullptr, *psf = nullptr;
    double *ca = nullptr, *cx = nullptr, *cy = nullptr, *cs = nullptr;
    int64_t *c_added = nullptr, *c_updated = nullptr;
    int64_t cap = 0;
    DevState *st = nullptr;
    DevState *st_host = nullptr;          // pinned mirror for reads
    int32_t *work = nullptr;
    asp_component *comp_out = nullptr;
    asp::FitGlobal *fg = nullptr;
    double *partials = nullptr;
    double *diag_out = nullptr;           // asp_eval_trial's reduced sums (first use)
    Params P{};
    int peak_grid = 1024, update_grid = 1024;
    int phase = 0;                        // 0 ready, 1 peak found, 2 fitted
    // kernel timing: event pairs around the launches of asp_run
    bool timing = false;
    std::vector<hipEvent_t> events;       // 2 per launch slot
    std::vector<int> ev_kind;             // kind of each recorded pair
    double t_ms[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t t_n[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // the proposal network (input-major layout) and training-sample recording
    float *net = nullptr;
    asp::NetParams netp{};
    double *sumsq = nullptr;              // 1024 partials, the total, the tracked read
    double *sq_slots = nullptr;           // per update work-group deltas of the sum of R^2
    unsigned long long *px_slots = nullptr;  // per update work-group pixel counts
    // the smoothing method's device buffers (allocated on first use)
    float *sm_vt = nullptr, *sm_taps = nullptr, *sm_w = nullptr, *sm_map = nullptr;
    unsigned long long *sm_keys = nullptr;
    int32_t *sm_dirty = nullptr, *sm_list = nullptr;
    unsigned int *sm_count = nullptr;
    // the incremental peak search's tile keys, flags and list
    unsigned long long *pk_keys = nullptr;
    int32_t *pk_dirty = nullptr;
    unsigned int *pk_count = nullptr;
    int pk_tiles = 0;                     // > 0: the incremental peak search is on
    // the exact-PSF refresh: the dirty image kept from creation, the padded
    // grid and spectra, the FFT plans (made on first use)
    float *dirty0 = nullptr;
    double *rf_grid = nullptr;
    double2 *rf_spec = nullptr, *rf_pspec = nullptr;
    hipfftHandle rf_fwd = 0, rf_inv = 0;
    bool rf_ready = false;
    asp::RefreshArgs rf{};
    // the Asp-Clean2004 iteration: four padded grids and spectra, partial
    // sums, the LM state and its pinned mirror, the batched inverse plan
    // (first use)
    double *a4_grid = nullptr, *a4_part = nullptr;
    double2 *a4_spec = nullptr;
    asp::A4State *a4_state = nullptr, *a4_host = nullptr;
    hipfftHandle a4_inv = 0;
    bool a4_ready = false;
    double *a4_taps = nullptr;            // per-axis factors of the rendering
    double2 *a4_fac = nullptr;            // their 1-D DFTs
    int32_t *a4_tapi = nullptr;
    int32_t a4_conv = 0;                  // 0 cheaper of direct / FFT, 1 FFT, 2 direct
    asp::A4Args a4{};
    float *model_dev = nullptr;           // asp_model_image's device copy (first use)
    bool in_batch = false;                // a field of an asp_batch
    std::string err;
};

namespace asp {
hipError_t launch_net_layout(const float *flat, float *net, hipStream_t s);
}

namespace {

asp_status fail(asp_ctx *c, asp_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_OR_FAIL(ctx, call)                                                         \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail((ctx), ASP_ERR_DEVICE,                                         \
                        std::string(#call ": ") + hipGetErrorString(e_));             \
    } while (0)

template <typename T>
hipError_t dev_alloc(T **p, size_t count)
{
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

void release(asp_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->R); (void)hipFree(c->psf);
    (void)hipFree(c->ca); (void)hipFree(c->cx); (void)hipFree(c->cy); (void)hipFree(c->cs);
    (void)hipFree(c->c_added); (void)hipFree(c->c_updated);
    (void)hipFree(c->st); (void)hipFree(c->work); (void)hipFree(c->comp_out);
    (void)hipFree(c->fg); (void)hipFree(c->partials); (void)hipFree(c->net);
    (void)hipFree(c->diag_out);
    (void)hipFree(c->sumsq);
    (void)hipFree(c->sq_slots);
    (void)hipFree(c->px_slots);
    (void)hipFree(c->sm_vt); (void)hipFree(c->sm_taps); (void)hipFree(c->sm_w);
    (void)hipFree(c->sm_map); (void)hipFree(c->sm_keys); (void)hipFree(c->sm_dirty);
    (void)hipFree(c->sm_list); (void)hipFree(c->sm_count);
    (void)hipFree(c->pk_keys); (void)hipFree(c->pk_dirty); (void)hipFree(c->pk_count);
    if (c->rf_fwd) (void)hipfftDestroy(c->rf_fwd);
    if (c->rf_inv) (void)hipfftDestroy(c->rf_inv);
    (void)hipFree(c->dirty0); (void)hipFree(c->rf_grid); (void)hipFree(c->rf_spec);
    (void)hipFree(c->rf_pspec);
    if (c->a4_inv) (void)hipfftDestroy(c->a4_inv);
    (void)hipFree(c->a4_grid); (void)hipFree(c->a4_part); (void)hipFree(c->a4_spec);
    (void)hipFree(c->a4_state);
    (void)hipFree(c->a4_taps); (void)hipFree(c->a4_tapi); (void)hipFree(c->a4_fac);
    if (c->a4_host) (void)hipHostFree(c->a4_host);
    (void)hipFree(c->model_dev);
    if (c->st_host) (void)hipHostFree(c->st_host);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// Copy a field range of the device state to the pinned mirror and wait.
asp_status pull_state(asp_ctx *c, size_t off, size_t len)
{
    HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st_host + off, (char *)c->st + off, len,
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status pull_all(asp_ctx *c) { return pull_state(c, 0, sizeof(DevState)); }

bool fit_setup_done = false;

// Waits between work-groups end after 2 s of device wall clock.
unsigned long long spin_limit_ticks(int device)
{
    int rate_khz = 100000;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;
    return (unsigned long long)rate_khz * 2000ull;
}

// The smoothing method's trial widths, taps and buffers (Sect. 2 step 1,
// Sect. 3).  Widths omega_b 2^j, j < smooth_scales, not above the fit's width
// bound; taps k(d) = exp(-(d - h)^2 / (2 sigma^2)), d = 0 .. 2h, rounded to
// FP32 and padded with zeros to whole blocks of kSmRb.
asp_status setup_smoothing(asp_ctx *c)
{
    if (c->sm_vt) return ASP_OK;
    const int64_t H = c->H, W = c->W, N = H * W;
    const double wb = c->st_host->omega_b;
    double cap = c->opt.max_width > 0.0 ? c->opt.max_width : (double)(H < W ? H : W) / 8.0;
    if (cap < wb) cap = wb;
    const int want = c->opt.smooth_scales == 0 ? 5 : c->opt.smooth_scales;
    asp::SmoothParams &S = c->P.sm;
    S = asp::SmoothParams{};
    std::vector<float> taps;
    int n = 0;
    for (int j = 0; j < want; ++j) {
        const double sig = wb * (double)(1 << j);
        if (j > 0 && sig > cap) break;
        const int h = asp::halfwidth(sig, c->opt.window_sigmas);
        const int nb = (2 * h + 1 + asp::kSmRb - 1) / asp::kSmRb;
        S.sig[n] = sig;
        S.h[n] = h;
        S.nb[n] = nb;
        S.off[n] = (int32_t)taps.size();
        for (int d = 0; d < nb * asp::kSmRb; ++d) {
            const double dd = (double)(d - h);
            taps.push_back(d <= 2 * h ? (float)exp(-(dd * dd) / (2.0 * sig * sig)) : 0.0f);
        }
        ++n;
    }
    if ((double)N * (double)n >= 4294967295.0)
        return fail(c, ASP_ERR_INVALID_ARG, "image too large for the smoothing method's keys");
    // norm factors 1 / sqrt(sum of k^2 over the clipped 1-D window), FP64
    std::vector<float> w((size_t)n * (W + H));
    for (int j = 0; j < n; ++j) {
        const int h = S.h[j];
        const double sig = S.sig[j];
        auto f = [&](int64_t pos, int64_t len) {
            double acc = 0.0;
            for (int d = -h; d <= h; ++d) {
                if (pos + d < 0 || pos + d >= len) continue;
                const double k = exp(-((double)d * d) / (2.0 * sig * sig));
                acc += k * k;
            }
            return (float)(1.0 / sqrt(acc));
        };
        for (int64_t x = 0; x < W; ++x) w[(size_t)j * W + x] = f(x, W);
        for (int64_t y = 0; y < H; ++y) w[(size_t)n * W + (size_t)j * H + y] = f(y, H);
    }
    S.n = n;
    S.norm = c->opt.smooth_norm;
    S.switch_area = c->opt.switch_area;
    S.tiles_x = (int32_t)((W + asp::kSmTile - 1) / asp::kSmTile);
    S.tiles_y = (int32_t)((H + asp::kSmTile - 1) / asp::kSmTile);
    const int64_t ntiles = (int64_t)S.tiles_x * S.tiles_y;
    S.map_scale = -1;
    auto bad = [&](hipError_t e) {
        (void)hipFree(c->sm_vt); (void)hipFree(c->sm_taps); (void)hipFree(c->sm_w);
        (void)hipFree(c->sm_keys); (void)hipFree(c->sm_dirty);
        (void)hipFree(c->sm_list); (void)hipFree(c->sm_count);
        c->sm_vt = c->sm_taps = c->sm_w = nullptr;
        c->sm_keys = nullptr;
        c->sm_dirty = c->sm_list = nullptr;
        c->sm_count = nullptr;
        S = asp::SmoothParams{};
        return fail(c, e == hipErrorOutOfMemory ? ASP_ERR_NOMEM : ASP_ERR_DEVICE,
                    std::string("smoothing buffers: ") + hipGetErrorString(e));
    };
    hipError_t e = dev_alloc(&c->sm_vt, (size_t)n * N);
    if (e == hipSuccess) e = dev_alloc(&c->sm_taps, taps.size());
    if (e == hipSuccess) e = dev_alloc(&c->sm_w, w.size());
    if (e == hipSuccess) e = dev_alloc(&c->sm_keys, (size_t)n * ntiles);
    if (e == hipSuccess) e = dev_alloc(&c->sm_dirty, (size_t)2 * n * ntiles);
    if (e == hipSuccess) e = dev_alloc(&c->sm_list, (size_t)2 * n * ntiles);
    if (e == hipSuccess) e = dev_alloc(&c->sm_count, 2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->sm_taps, taps.data(), sizeof(float) * taps.size(),
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->sm_w, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->sm_keys, 0, sizeof(unsigned long long) * n * ntiles, c->stream);
    if (e != hipSuccess) return bad(e);
    S.vt = c->sm_vt;
    S.taps = c->sm_taps;
    S.wx = c->sm_w;
    S.wy = c->sm_w + (size_t)n * W;
    S.keys = c->sm_keys;
    S.dirty_a = c->sm_dirty;
    S.dirty_b = c->sm_dirty + (size_t)n * ntiles;
    S.list_a = c->sm_list;
    S.list_b = c->sm_list + (size_t)n * ntiles;
    S.count = c->sm_count;
    // every tile stale
    e = asp::launch_smooth_mark_all(c->P, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bad(e);
    return ASP_OK;
}

// Init mode 2: buffers, every tile stale, and the next iteration smooths.
asp_status enter_smoothing(asp_ctx *c)
{
    const bool fresh = c->sm_vt == nullptr;
    asp_status s = setup_smoothing(c);
    if (s != ASP_OK) return s;
    if (!fresh) HIP_OR_FAIL(c, asp::launch_smooth_mark_all(c->P, c->stream));
    DevState *h = c->st_host;
    h->smooth_now = 1;
    h->smooth_ready = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st + offsetof(DevState, smooth_now), &h->smooth_now,
                                  2 * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->P.smooth = 1;
    return ASP_OK;
}

asp_status create_common(const float *dirty, bool dirty_dev, int64_t H, int64_t W,
                         const float *psf, bool psf_dev, int64_t Hp, int64_t Wp, float gain,
                         float threshold, const asp_options *opt_in, asp_ctx **out)
{
    if (!out) return ASP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!dirty || !psf || H <= 0 || W <= 0 || Hp <= 0 || Wp <= 0) return ASP_ERR_INVALID_ARG;
    if ((double)H * (double)W >= 4294967295.0) return ASP_ERR_INVALID_ARG;
    if (!(gain > 0.0f && gain <= 1.0f) || !(threshold >= 0.0f) || !isfinite(threshold))
        return ASP_ERR_INVALID_ARG;
    asp_options opt;
    asp_default_options(&opt);
    if (opt_in) {
        if (opt_in->struct_size != (int32_t)sizeof(asp_options)) return ASP_ERR_INVALID_ARG;
        opt = *opt_in;
    }
    if (opt.max_iter < 0 || opt.max_active < 1 || opt.max_active > ASP_MAX_ACTIVE ||
        opt.lm_max_iter < 1 || opt.init_mode < 0 || opt.init_mode > 2 || opt.capacity < 0 ||
        opt.smooth_scales < 0 || opt.smooth_scales > ASP_MAX_SCALES || opt.smooth_norm < 0 ||
        opt.smooth_norm > 1 || opt.switch_area < 0 || opt.switch_area > 1 || opt.peak_tiles < 0 ||
        opt.peak_tiles > 1 || opt.refresh_every < 0 || opt.update_launch < 0 ||
        opt.update_launch > 1 || opt.reserved != 0 ||
        opt.fit_solo_tiles < -1 || opt.fit_min_tiles < 0 || opt.fit_group < 0 ||
        !(opt.window_sigmas > 0.0) || !(opt.max_width >= 0.0) || !(opt.lm_mu0 > 0.0) ||
        !(opt.lm_tol > 0.0) || !(opt.psf_lobe_frac > 0.0 && opt.psf_lobe_frac < 1.0))
        return ASP_ERR_INVALID_ARG;

    asp_ctx *c = new (std::nothrow) asp_ctx();
    if (!c) return ASP_ERR_NOMEM;
    c->H = H; c->W = W; c->Hp = Hp; c->Wp = Wp; c->opt = opt;
    c->cap = opt.capacity > 0 ? opt.capacity : (opt.max_iter > 0 ? opt.max_iter : 1);
    const int64_t n = H * W, np = Hp * Wp;
    auto bail = [&](asp_status s) {
        std::string msg = c->err;
        release(c);
        delete c;
        fprintf(stderr, "asp_create: %s\n", msg.c_str());
        return s;
    };
#define CREATE_HIP(call)                                                               \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            c->err = std::string(#call ": ") + hipGetErrorString(e_);                 \
            return bail(e_ == hipErrorOutOfMemory ? ASP_ERR_NOMEM : ASP_ERR_DEVICE);  \
        }                                                                              \
    } while (0)

    CREATE_HIP(hipGetDevice(&c->device));
    if (opt.stream) {
        c->stream = (hipStream_t)opt.stream;
    } else {
        CREATE_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    if (!fit_setup_done) {
        CREATE_HIP(asp::fit_kernel_setup());
        fit_setup_done = true;
    }
    CREATE_HIP(dev_alloc(&c->R, n));
    CREATE_HIP(dev_alloc(&c->dirty0, n));
    CREATE_HIP(dev_alloc(&c->psf, np));
    CREATE_HIP(dev_alloc(&c->ca, c->cap));
    CREATE_HIP(dev_alloc(&c->cx, c->cap));
    CREATE_HIP(dev_alloc(&c->cy, c->cap));
    CREATE_HIP(dev_alloc(&c->cs, c->cap));
    CREATE_HIP(dev_alloc(&c->c_added, c->cap));
    CREATE_HIP(dev_alloc(&c->c_updated, c->cap));
    CREATE_HIP(dev_alloc(&c->st, 1));
    CREATE_HIP(dev_alloc(&c->sumsq, 1026));
    CREATE_HIP(dev_alloc(&c->sq_slots, asp::kSqSlots));
    CREATE_HIP(dev_alloc(&c->px_slots, asp::kSqSlots));
    CREATE_HIP(hipMemsetAsync(c->px_slots, 0, sizeof(unsigned long long) * asp::kSqSlots,
                              c->stream));
    CREATE_HIP(dev_alloc(&c->work, np > 2 ? np : 2));
    const int fit_grid = asp::fit_grid_size(c->device);
    if (fit_grid < 1) {
        c->err = "the fit kernel's work-groups cannot all be resident at once (private segment "
                 "or no occupancy): its cooperative launch is refused";
        return bail(ASP_ERR_DEVICE);
    }
    CREATE_HIP(dev_alloc(&c->fg, 1));
    CREATE_HIP(dev_alloc(&c->partials, (size_t)(fit_grid + asp::kMaxGroups) * asp::kPartStride));
    CREATE_HIP(hipMemsetAsync(c->fg, 0, sizeof(asp::FitGlobal), c->stream));
    CREATE_HIP(hipHostMalloc((void **)&c->st_host, sizeof(DevState), hipHostMallocDefault));

    const hipMemcpyKind kd = dirty_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kp = psf_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    CREATE_HIP(hipMemcpyAsync(c->R, dirty, sizeof(float) * n, kd, c->stream));
    CREATE_HIP(hipMemcpyAsync(c->dirty0, dirty, sizeof(float) * n, kd, c->stream));
    CREATE_HIP(hipMemcpyAsync(c->psf, psf, sizeof(float) * np, kp, c->stream));
    memset(c->st_host, 0, sizeof(DevState));
    c->st_host->forced_idx = -1;
    c->st_host->sq_slots = c->sq_slots;
    c->st_host->sq_nslots = asp::kSqSlots;
    c->st_host->px_slots = c->px_slots;
    CREATE_HIP(hipMemcpyAsync(c->st, c->st_host, sizeof(DevState), hipMemcpyHostToDevice,
                              c->stream));
    // NaN / Inf in either image is an error (no CPU scan: a device kernel).
    CREATE_HIP(hipMemsetAsync(c->work, 0, 2 * sizeof(int32_t), c->stream));
    CREATE_HIP(asp::launch_check_finite(c->R, n, c->work, c->stream));
    CREATE_HIP(asp::launch_check_finite(c->psf, np, c->work + 1, c->stream));
    int32_t flags[2] = {0, 0};
    CREATE_HIP(hipMemcpyAsync(flags, c->work, sizeof(flags), hipMemcpyDeviceToHost, c->stream));
    CREATE_HIP(hipStreamSynchronize(c->stream));
    if (flags[0] || flags[1]) {
        c->err = flags[0] ? "dirty image holds NaN or Inf" : "PSF holds NaN or Inf";
        return bail(ASP_ERR_NONFINITE);
    }
    // the tracked sum of R^2 starts from a full pass over the dirty image
    CREATE_HIP(asp::launch_sumsq(c->R, n, c->sumsq, 1024, c->sumsq + 1024, c->stream));
    CREATE_HIP(asp::launch_sq_rebase(c->st, c->sumsq + 1024, c->stream));
    CREATE_HIP(asp::launch_psf_fit(c->psf, Hp, Wp, opt.psf_lobe_frac, c->st, c->work, c->stream));
    CREATE_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost,
                              c->stream));
    CREATE_HIP(hipStreamSynchronize(c->stream));
    if (c->st_host->psf_status != 0 || !(c->st_host->omega_b > 0.0) ||
        !isfinite(c->st_host->alpha_b)) {
        c->err = "PSF peak is not positive or its main lobe cannot be fitted";
        return bail(ASP_ERR_PSF);
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    const int64_t n4 = n / 4;
    int64_t pg = cus * 8;
    int64_t need = (n4 + 255) / 256;
    c->peak_grid = (int)(need < pg ? (need > 0 ? need : 1) : pg);
    // one slot of the tracked sum of R^2 per update work-group
    c->update_grid = cus * 8 < asp::kSqSlots ? cus * 8 : asp::kSqSlots;

    Params &P = c->P;
    P.R = c->R; P.H = H; P.W = W;
    P.ca = c->ca; P.cx = c->cx; P.cy = c->cy; P.cs = c->cs;
    P.c_added = c->c_added; P.c_updated = c->c_updated;
    P.cap = c->cap;
    P.st = c->st;
    P.gain = (double)gain;
    P.threshold = (double)threshold;
    P.max_iter = opt.max_iter;
    P.max_active = opt.max_active;
    P.lm_max_iter = opt.lm_max_iter;
    P.window_sigmas = opt.window_sigmas;
    P.max_width = opt.max_width;
    P.lm_mu0 = opt.lm_mu0;
    P.lm_tol = opt.lm_tol;
    P.use_proposal = 1;
    P.fit_grid = fit_grid;
    P.solo_tiles = opt.fit_solo_tiles == 0 ? 16 : opt.fit_solo_tiles;
    P.min_tiles = opt.fit_min_tiles == 0 ? 2 : opt.fit_min_tiles;
    P.spin_ticks = spin_limit_ticks(c->device);
    P.group = opt.fit_group == 0 ? 16 : opt.fit_group;
    if ((fit_grid + P.group - 1) / P.group > asp::kMaxGroups) {
        c->err = "fit_group too small for the grid";
        return bail(ASP_ERR_INVALID_ARG);
    }
    P.fg = c->fg;
    P.partials = c->partials;
    if (opt.init_mode == 2) {
        asp_status s = enter_smoothing(c);
        if (s != ASP_OK) return bail(s);
    }
    if (opt.peak_tiles) {
        // the buffers live in the device state; every tile stale: the first
        // search scans the whole image
        asp::PeakTiles &K = c->st_host->pk;
        K.tiles_x = (int32_t)((W + asp::kPkTile - 1) / asp::kPkTile);
        K.tiles_y = (int32_t)((H + asp::kPkTile - 1) / asp::kPkTile);
        const size_t nt = (size_t)K.tiles_x * K.tiles_y;
        CREATE_HIP(dev_alloc(&c->pk_keys, nt));
        CREATE_HIP(dev_alloc(&c->pk_dirty, 2 * nt));
        CREATE_HIP(dev_alloc(&c->pk_count, 1));
        K.keys = c->pk_keys;
        K.dirty = c->pk_dirty;
        K.list = c->pk_dirty + nt;
        K.count = c->pk_count;
        CREATE_HIP(hipMemcpyAsync((char *)c->st + offsetof(DevState, pk), &K, sizeof(K),
                                  hipMemcpyHostToDevice, c->stream));
        CREATE_HIP(asp::launch_peak_mark_all(P, c->stream));
        CREATE_HIP(hipStreamSynchronize(c->stream));
        c->pk_tiles = (int)nt;
    }
    *out = c;
    return ASP_OK;
#undef CREATE_HIP
}

asp_status stop_status(const asp_ctx *c)
{
    int32_t s = c->st_host->stop;
    if (s == ASP_STOP_THRESHOLD || s == ASP_STOP_MAXITER) return (asp_status)s;
    if (s < 0) return (asp_status)s;
    return ASP_OK;
}

// Timed launch: an event pair around the launch when timing is on.
template <typename F>
asp_status timed(asp_ctx *c, int kind, F launch)
{
    if (!c->timing) {
        HIP_OR_FAIL(c, launch());
        return ASP_OK;
    }
    const size_t slot = c->ev_kind.size();
    while (c->events.size() < 2 * (slot + 1)) {
        hipEvent_t e;
        HIP_OR_FAIL(c, hipEventCreate(&e));
        c->events.push_back(e);
    }
    HIP_OR_FAIL(c, hipEventRecord(c->events[2 * slot], c->stream));
    HIP_OR_FAIL(c, launch());
    HIP_OR_FAIL(c, hipEventRecord(c->events[2 * slot + 1], c->stream));
    c->ev_kind.push_back(kind);
    return ASP_OK;
}

// Fold the recorded pairs into the per-kind totals (the stream has drained).
asp_status harvest(asp_ctx *c)
{
    for (size_t i = 0; i < c->ev_kind.size(); ++i) {
        float ms = 0.0f;
        HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->events[2 * i], c->events[2 * i + 1]));
        c->t_ms[c->ev_kind[i]] += (double)ms;
        c->t_n[c->ev_kind[i]] += 1;
    }
    c->ev_kind.clear();
    return ASP_OK;
}

bool use_net(const asp_ctx *c) { return c->opt.init_mode == 1 && c->net; }

// The smallest size >= n whose prime factors are 2, 3, 5 and 7 (fast FFTs).
int64_t fft_size(int64_t n)
{
    for (int64_t m = n > 1 ? n : 1;; ++m) {
        int64_t r = m;
        for (int64_t f : {2, 3, 5, 7})
            while (r % f == 0) r /= f;
        if (r == 1) return m;
    }
}

const char *fft_text(hipfftResult r)
{
    return r == HIPFFT_SUCCESS ? "ok" : "hipFFT call failed";
}

// Buffers, plans and the PSF's spectrum of the exact-PSF refresh (first use).
asp_status setup_refresh(asp_ctx *c)
{
    if (c->rf_ready) return ASP_OK;
    const int64_t H = c->H, W = c->W, Hp = c->Hp, Wp = c->Wp;
    std::vector<float> ph((size_t)(Hp * Wp));
    HIP_OR_FAIL(c, hipMemcpyAsync(ph.data(), c->psf, sizeof(float) * ph.size(),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    size_t best = 0;                        // the peak pixel: largest value, lowest index
    for (size_t i = 1; i < ph.size(); ++i)
        if (ph[i] > ph[best]) best = i;
    const int64_t Py = fft_size(H + Hp - 1), Px = fft_size(W + Wp - 1);
    const size_t nspec = (size_t)Py * (size_t)(Px / 2 + 1);
    // a call after a failed one keeps what that one allocated
    if (!c->rf_grid) HIP_OR_FAIL(c, dev_alloc(&c->rf_grid, (size_t)(Py * Px)));
    if (!c->rf_spec) HIP_OR_FAIL(c, dev_alloc(&c->rf_spec, nspec));
    if (!c->rf_pspec) HIP_OR_FAIL(c, dev_alloc(&c->rf_pspec, nspec));
    hipfftResult r = HIPFFT_SUCCESS;
    if (!c->rf_fwd) r = hipfftPlan2d(&c->rf_fwd, (int)Py, (int)Px, HIPFFT_D2Z);
    if (r == HIPFFT_SUCCESS && !c->rf_inv) r = hipfftPlan2d(&c->rf_inv, (int)Py, (int)Px, HIPFFT_Z2D);
    if (r == HIPFFT_SUCCESS) r = hipfftSetStream(c->rf_fwd, c->stream);
    if (r == HIPFFT_SUCCESS) r = hipfftSetStream(c->rf_inv, c->stream);
    if (r != HIPFFT_SUCCESS) return fail(c, ASP_ERR_DEVICE, std::string("refresh plans: ") + fft_text(r));
    asp::RefreshArgs &a = c->rf;
    a.dirty = c->dirty0;
    a.psf = c->psf;
    a.R = c->R;
    a.ca = c->ca; a.cx = c->cx; a.cy = c->cy; a.cs = c->cs;
    a.st = c->st;
    a.grid = c->rf_grid;
    a.spec = c->rf_spec;
    a.pspec = c->rf_pspec;
    a.H = H; a.W = W; a.Hp = Hp; a.Wp = Wp; a.Py = Py; a.Px = Px;
    a.ci = (int32_t)(best / (size_t)Wp);
    a.cj = (int32_t)(best % (size_t)Wp);
    a.window_sigmas = c->opt.window_sigmas;
    a.force = 1;
    HIP_OR_FAIL(c, asp::refresh_psf_spectrum(a, &c->rf_fwd, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->rf_ready = true;
    return ASP_OK;
}

// A full pass over R re-bases the tracked sum of R^2 (after every change of R
// that is not a windowed update).
asp_status rebase_sumsq(asp_ctx *c)
{
    HIP_OR_FAIL(c, asp::launch_sumsq(c->R, c->H * c->W, c->sumsq, 1024, c->sumsq + 1024,
                                     c->stream));
    HIP_OR_FAIL(c, asp::launch_sq_rebase(c->st, c->sumsq + 1024, c->stream));
    return ASP_OK;
}

// The pixels rewritten by all updates so far (sum of the per work-group counts),
// with the rest of the device state pulled to the host.
asp_status pull_with_px(asp_ctx *c, unsigned long long *px)
{
    HIP_OR_FAIL(c, asp::launch_px_read(c->st, c->stream));
    asp_status s = pull_all(c);
    if (s == ASP_OK && px) *px = c->st_host->px_total;
    return s;
}

// One refresh on the stream; then every tile of the incremental searches is
// stale and the tracked sum of R^2 is re-based (the whole residual changed).
asp_status enqueue_refresh(asp_ctx *c, int force)
{
    asp::RefreshArgs a = c->rf;
    a.force = force;
    asp_status s = timed(c, 6, [&] {
        return asp::refresh_residual(a, &c->rf_fwd, &c->rf_inv, c->stream);
    });
    if (s != ASP_OK) return s;
    if (c->pk_tiles) HIP_OR_FAIL(c, asp::launch_peak_mark_all(c->P, c->stream));
    if (c->P.sm.n > 0) HIP_OR_FAIL(c, asp::launch_smooth_mark_all(c->P, c->stream));
    return rebase_sumsq(c);
}

asp_status enqueue_iteration(asp_ctx *c)
{
    if (c->opt.init_mode == 1 && !c->net)
        return fail(c, ASP_ERR_STATE, "learned start values need a network (asp_set_mlp)");
    asp_status s = timed(c, 0, [&] {
        return c->pk_tiles ? asp::launch_peak_tiles(c->P, c->pk_tiles, c->stream)
                           : asp::launch_peak(c->P, c->peak_grid, c->stream);
    });
    if (s == ASP_OK && c->P.smooth)
        s = timed(c, 4, [&] { return asp::launch_smooth_passes(c->P, 0, c->stream); });
    if (s == ASP_OK && c->P.smooth)
        s = timed(c, 5, [&] { return asp::launch_smooth_pick(c->P, 0, c->stream); });
    if (s == ASP_OK && (use_net(c) || c->P.rec_cap > 0))
        s = timed(c, 3, [&] {
            return asp::launch_propose(c->P, c->netp, use_net(c) ? 1 : 0, c->stream);
        });
    // the fit kernel's work-groups take the update after the commit, unless
    // the options ask for its own launch
    asp::Params q = c->P;
    q.fuse_update = c->opt.update_launch == 0 ? 1 : 0;
    if (s == ASP_OK) s = timed(c, 1, [&] { return asp::launch_fit(q, c->stream); });
    if (s == ASP_OK && !q.fuse_update)
        s = timed(c, 2, [&] { return asp::launch_update(c->P, c->update_grid, c->stream); });
    return s;
}


// Buffers and the batched inverse plan of the Asp-Clean2004 iteration (first
// use); the PSF's spectrum, its peak pixel and the single inverse plan are the
// refresh's.
asp_status setup_2004(asp_ctx *c)
{
    if (c->a4_ready) return ASP_OK;
    asp_status s = setup_refresh(c);
    if (s == ASP_OK) s = setup_smoothing(c);
    if (s != ASP_OK) return s;
    const asp::RefreshArgs &r = c->rf;
    const int64_t Py = r.Py, Px = r.Px;
    const size_t plane = (size_t)(Py * Px), nspec = (size_t)Py * (size_t)(Px / 2 + 1);
    // a call after a failed one keeps what that one allocated
    hipError_t e = hipSuccess;
    if (!c->a4_grid) e = dev_alloc(&c->a4_grid, 4 * plane);
    if (e == hipSuccess && !c->a4_spec) e = dev_alloc(&c->a4_spec, 4 * nspec);
    if (e == hipSuccess && !c->a4_part)
        e = dev_alloc(&c->a4_part, (size_t)asp::kA4Blocks * asp::kA4Sums);
    if (e == hipSuccess && !c->a4_state) e = dev_alloc(&c->a4_state, 1);
    if (e == hipSuccess && !c->a4_host) e = hipHostMalloc((void **)&c->a4_host, sizeof(asp::A4State));
    if (e == hipSuccess && !c->a4_taps) e = dev_alloc(&c->a4_taps, (size_t)(3 * (c->H + c->W)));
    if (e == hipSuccess && !c->a4_tapi) e = dev_alloc(&c->a4_tapi, 4);
    if (e == hipSuccess && !c->a4_fac) e = dev_alloc(&c->a4_fac, (size_t)(3 * (Py + Px / 2 + 1)));
    if (e != hipSuccess)
        return fail(c, e == hipErrorOutOfMemory ? ASP_ERR_NOMEM : ASP_ERR_DEVICE,
                    std::string("Asp-Clean2004 buffers: ") + hipGetErrorString(e));
    HIP_OR_FAIL(c, hipMemsetAsync(c->a4_state, 0, sizeof(asp::A4State), c->stream));
    int n[2] = {(int)Py, (int)Px};
    hipfftResult fr = HIPFFT_SUCCESS;
    if (!c->a4_inv)
        fr = hipfftPlanMany(&c->a4_inv, 2, n, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_Z2D, 4);
    if (fr == HIPFFT_SUCCESS) fr = hipfftSetStream(c->a4_inv, c->stream);
    if (fr != HIPFFT_SUCCESS)
        return fail(c, ASP_ERR_DEVICE, std::string("Asp-Clean2004 plans: ") + fft_text(fr));
    asp::A4Args &a = c->a4;
    a.R = c->R;
    a.st = c->st;
    a.s = c->a4_state;
    a.ca = c->ca; a.cx = c->cx; a.cy = c->cy; a.cs = c->cs;
    a.c_added = c->c_added; a.c_updated = c->c_updated;
    a.cap = c->cap;
    a.grid = c->a4_grid;
    a.spec = c->a4_spec;
    a.pspec = r.pspec;
    a.partials = c->a4_part;
    a.psf = c->psf;
    a.taps = c->a4_taps;
    a.fac = c->a4_fac;
    a.tapi = c->a4_tapi;
    a.grid_cap = 4 * (int64_t)plane;
    a.Hp = c->Hp; a.Wp = c->Wp;
    a.H = c->H; a.W = c->W; a.Py = Py; a.Px = Px;
    a.ci = r.ci; a.cj = r.cj;
    a.budget = c->opt.lm_max_iter;
    a.nblk = (int32_t)(c->H < asp::kA4Blocks ? c->H : asp::kA4Blocks);
    a.gain = c->P.gain;
    a.window_sigmas = c->opt.window_sigmas;
    const double wb = c->st_host->omega_b;
    double smax = c->opt.max_width > 0.0 ? c->opt.max_width : (double)(c->H < c->W ? c->H : c->W) / 8.0;
    a.s_max = smax > wb ? smax : wb;
    a.mu0 = c->opt.lm_mu0;
    a.tol = c->opt.lm_tol;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->a4_ready = true;
    return ASP_OK;
}

// The direct convolution's multiply-add slots that take about as long as the
// FFT route per padded pixel: an evaluation (factor DFTs, spectral product,
// batched inverse transform, sums) and the update (one inverse transform).
constexpr double kA4FftEval = 1000.0, kA4FftUpdate = 250.0;

// Taps per axis of the rendering at squared width v: 12 for the narrow
// rendering, 2 h + 1 for the sampled Gaussian (at least 12 either way, so the
// count grows with v), clipped to the image by the caller.
int64_t a4_taps_bound(const asp_ctx *c, double v)
{
    const double om = sqrt(v > 0.0 ? v : 0.0);
    const int64_t n = om >= 1.0 ? 2 * (int64_t)asp::halfwidth(om, c->opt.window_sigmas) + 1 : 12;
    return n < 12 ? 12 : n;
}

// Whether an Asp-Clean2004 evaluation (planes 3) or update (planes 1)
// convolves directly.  v_cap bounds the squared width of every point the
// launches may meet: at that width the row pass's (H + nr - 1) x W rows per
// factor must fit the grids.  v is the width of the point itself: by default
// the direct route's multiply-add slots, planes nc (H + nr - 1) W for the row
// pass and (5 or 1) (nr + 3) H W for the column pass, must undercut
// kA4FftEval (kA4FftUpdate) per padded pixel.
bool a4_direct(const asp_ctx *c, double v, double v_cap, int planes)
{
    if (c->a4_conv == 1) return false;
    const double H = (double)c->H, W = (double)c->W;
    const double padded = (double)c->rf.Py * (double)c->rf.Px;
    const double ncap = (double)std::min(a4_taps_bound(c, v_cap), c->H);
    if ((double)planes * (H + ncap - 1.0) * W > 4.0 * padded) return false;
    if (c->a4_conv == 2) return true;
    const double nr = (double)std::min(a4_taps_bound(c, v), c->H);
    const double nc = (double)std::min(a4_taps_bound(c, v), c->W);
    const double slots = (double)planes * nc * (H + nr - 1.0) * W +
                         (planes == 3 ? 5.0 : 1.0) * (nr + 3.0) * H * W;
    return slots <= (planes == 3 ? kA4FftEval : kA4FftUpdate) * padded;
}

asp_status pull_a4(asp_ctx *c)
{
    HIP_OR_FAIL(c, hipMemcpyAsync(c->a4_host, c->a4_state, sizeof(asp::A4State),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

// One Asp-Clean2004 iteration: the peak and the stop test, the smoothing
// start, LM evaluations of Eq. 3 until the fit ends (the host reads the
// device's LM state after each), the exact update and the new component.
asp_status step_2004(asp_ctx *c, asp_fit2004_report *rep)
{
    asp_status s = setup_2004(c);
    if (s == ASP_OK) s = pull_all(c);
    if (s != ASP_OK) return s;
    s = stop_status(c);
    if (s != ASP_OK) return s;
    s = timed(c, 0, [&] {
        return c->pk_tiles ? asp::launch_peak_tiles(c->P, c->pk_tiles, c->stream)
                           : asp::launch_peak(c->P, c->peak_grid, c->stream);
    });
    if (s == ASP_OK) HIP_OR_FAIL(c, asp::launch_peak_decode(c->P, c->stream));
    if (s == ASP_OK) s = timed(c, 4, [&] { return asp::launch_smooth_passes(c->P, 1, c->stream); });
    if (s == ASP_OK) s = timed(c, 5, [&] { return asp::launch_smooth_pick(c->P, 1, c->stream); });
    if (s == ASP_OK) HIP_OR_FAIL(c, asp::a4_begin(c->a4, c->stream));
    if (s == ASP_OK) s = pull_all(c);
    if (s == ASP_OK) s = pull_a4(c);
    if (s != ASP_OK) return s;
    const DevState *h = c->st_host;
    if (h->stop) {
        s = harvest(c);
        return s != ASP_OK ? s : stop_status(c);
    }
    // Every evaluation either ends the fit or spends a trial of the budget, so
    // at most budget + 1 are needed.  On small grids, where an evaluation
    // costs less than the host's round trip, four are queued between reads of
    // the LM state; those queued after the end return at once (their FFTs
    // inverse-transform stale spectra).  The convolution is chosen per read,
    // by the squared width of the next point; when four are queued, the fit
    // bound on that width must also let the direct route fit the grids.
    const int per_read = c->rf.Py * c->rf.Px <= (int64_t)1024 * 1024 ? 4 : 1;
    int32_t direct_evals = 0;
    for (int32_t queued = 0; !c->a4_host->done;) {
        if (queued >= c->a4.budget + 1)
            return fail(c, ASP_ERR_STATE, "the Asp-Clean2004 fit did not end within its budget");
        const bool direct = a4_direct(c, c->a4_host->te[3],
                                      per_read == 1 ? c->a4_host->te[3] : c->a4_host->hi[3], 3);
        const int32_t evals0 = c->a4_host->evals;
        for (int b = 0; b < per_read && queued < c->a4.budget + 1; ++b, ++queued) {
            s = timed(c, 7, [&] {
                return direct ? asp::a4_trial_direct(c->a4, c->stream)
                              : asp::a4_trial(c->a4, &c->a4_inv, c->stream);
            });
            if (s != ASP_OK) return s;
        }
        s = pull_a4(c);
        if (s != ASP_OK) return s;
        if (direct) direct_evals += c->a4_host->evals - evals0;
    }
    const bool direct_up = a4_direct(c, c->a4_host->theta[3], c->a4_host->theta[3], 1);
    s = timed(c, 8, [&] {
        return direct_up ? asp::a4_commit_direct(c->a4, c->stream)
                         : asp::a4_commit(c->a4, &c->rf_inv, c->stream);
    });
    if (s != ASP_OK) return s;
    if (c->pk_tiles) HIP_OR_FAIL(c, asp::launch_peak_mark_all(c->P, c->stream));
    HIP_OR_FAIL(c, asp::launch_smooth_mark_all(c->P, c->stream));
    s = rebase_sumsq(c);
    if (s == ASP_OK) s = pull_all(c);
    if (s == ASP_OK) s = harvest(c);
    if (s != ASP_OK) return s;
    const asp::A4State *a = c->a4_host;
    if (rep) {
        memset(rep, 0, sizeof *rep);
        rep->idx = h->idx;
        rep->peak = h->peak;
        rep->trials = a->trials;
        rep->converged = a->converged;
        rep->evaluations = a->evals;
        rep->direct_evals = direct_evals;
        rep->direct_update = direct_up ? 1 : 0;
        for (int i = 0; i < 4; ++i) {
            rep->start[i] = h->smooth_start[i];
            rep->theta0[i] = a->theta0[i];
            rep->theta[i] = a->theta[i];
            rep->lo[i] = a->lo[i];
            rep->hi[i] = a->hi[i];
        }
        rep->chi2_init = a->chi2_init;
        rep->chi2_final = a->chi2;
        rep->scale = h->smooth_scale;
    }
    s = stop_status(c);
    if (s != ASP_OK) return s;
    return a->converged ? ASP_OK : ASP_LM_NOT_CONVERGED;
}

// The checkpoint blob: this header, then R (H x W FP32), then the component
// list (a, x, y, s as L doubles each, then iteration added and updated as L
// int64 each), all in host byte order.
struct StateHeader {
    char magic[8];
    int64_t H, W, k, L;
    int32_t smooth_now, reserved;
    double alpha_b, omega_b;
};
constexpr char kStateMagic[8] = {'A', 'S', 'P', 'S', 'T', 'A', 'T', '1'};

int64_t state_bytes(int64_t H, int64_t W, int64_t L)
{
    return (int64_t)sizeof(StateHeader) + 4 * H * W + 48 * L;
}
}  // namespace

// The report of the last fit from the host mirror of the device state.
void fill_report(const DevState *h, asp_fit_report *rep)
{
    memset(rep, 0, sizeof *rep);
    rep->n_active = h->n_active;
    for (int i = 0; i < h->n_active; ++i) rep->members[i] = h->members[i];
    rep->lm_iters = h->lm_iters;
    rep->converged = h->converged;
    rep->used_fallback = h->used_fallback;
    rep->idx = h->idx;
    rep->peak = h->peak;
    rep->chi2_init = h->chi2_init;
    rep->chi2_final = h->chi2_final;
    for (int i = 0; i < 4 * h->n_active; ++i) {
        rep->theta0[i] = h->theta0[i];
        rep->theta[i] = h->theta[i];
    }
    rep->fit_px = h->fit_px;
    rep->init_source = h->init_source;
    rep->start_from_proposal = h->start_prop;
    for (int i = 0; i < 4; ++i) rep->init[i] = h->init[i];
    rep->added = h->added;
}

extern "C" {

asp_status asp_default_options(asp_options *opt)
{
    if (!opt) return ASP_ERR_INVALID_ARG;
    memset(opt, 0, sizeof *opt);
    opt->struct_size = (int32_t)sizeof(asp_options);
    opt->max_iter = 1000;
    opt->max_active = 5;
    opt->lm_max_iter = 100;
    opt->init_mode = 0;
    opt->capacity = 0;
    opt->window_sigmas = 5.0;
    opt->max_width = 0.0;
    opt->lm_mu0 = 1e-3;
    opt->lm_tol = 1e-5;
    opt->psf_lobe_frac = 0.35;
    opt->stream = nullptr;
    return ASP_OK;
}

asp_status asp_create(const float *dirty, int64_t H, int64_t W, const float *psf, int64_t Hp,
                      int64_t Wp, float gain, float threshold, const asp_options *opt,
                      asp_ctx **out)
{
    return create_common(dirty, false, H, W, psf, false, Hp, Wp, gain, threshold, opt, out);
}

asp_status asp_create_device(const float *dirty_dev, int64_t H, int64_t W, const float *psf_dev,
                             int64_t Hp, int64_t Wp, float gain, float threshold,
                             const asp_options *opt, asp_ctx **out)
{
    return create_common(dirty_dev, true, H, W, psf_dev, true, Hp, Wp, gain, threshold, opt, out);
}

void asp_destroy(asp_ctx *ctx)
{
    release(ctx);
    delete ctx;
}

const char *asp_last_error(const asp_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

asp_status asp_find_peak(asp_ctx *c, int64_t *idx, float *value)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    asp_status ts = timed(c, 0, [&] {
        return c->pk_tiles ? asp::launch_peak_tiles(c->P, c->pk_tiles, c->stream)
                           : asp::launch_peak(c->P, c->peak_grid, c->stream);
    });
    if (ts != ASP_OK) return ts;
    HIP_OR_FAIL(c, asp::launch_peak_decode(c->P, c->stream));
    if (c->P.smooth) {
        HIP_OR_FAIL(c, asp::launch_smooth_passes(c->P, 0, c->stream));
        HIP_OR_FAIL(c, asp::launch_smooth_pick(c->P, 0, c->stream));
    }
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    s = harvest(c);
    if (s != ASP_OK) return s;
    if (idx) *idx = c->st_host->idx;
    if (value) *value = c->st_host->peak;
    s = stop_status(c);
    c->phase = (s == ASP_OK) ? 1 : 0;
    return s;
}

asp_status asp_fit_active_set(asp_ctx *c, int64_t idx, const asp_gauss *init,
                              asp_fit_report *rep)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->phase != 1) return fail(c, ASP_ERR_STATE, "asp_fit_active_set needs asp_find_peak first");
    if (idx < 0 || idx >= c->H * c->W) return fail(c, ASP_ERR_INVALID_ARG, "idx out of range");
    DevState *h = c->st_host;
    h->forced_idx = idx;
    HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st + offsetof(DevState, forced_idx), &h->forced_idx,
                                  sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    if (!init && c->opt.init_mode == 1 && !c->net)
        return fail(c, ASP_ERR_STATE, "learned start values need a network (asp_set_mlp)");
    if (init) {
        h->have_proposal = 1;
        h->proposal[0] = init->amp; h->proposal[1] = init->x;
        h->proposal[2] = init->y; h->proposal[3] = init->width;
        HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st + offsetof(DevState, have_proposal),
                                      &h->have_proposal,
                                      offsetof(DevState, n_active) - offsetof(DevState, have_proposal),
                                      hipMemcpyHostToDevice, c->stream));
    }
    const bool net_start = !init && use_net(c);
    if (net_start || c->P.rec_cap > 0)
        HIP_OR_FAIL(c, asp::launch_propose(c->P, c->netp, net_start ? 1 : 0, c->stream));
    HIP_OR_FAIL(c, asp::launch_fit(c->P, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    asp_status st = stop_status(c);
    if (st != ASP_OK) { c->phase = 0; return st; }
    if (rep) fill_report(h, rep);
    c->phase = 2;
    return h->converged ? ASP_OK : ASP_LM_NOT_CONVERGED;
}

asp_status asp_eval_trial(asp_ctx *c, int32_t m, const double *theta, const double *stored,
                          double *jtj, double *jtr, double *F, double *chi2, int64_t *npx)
{
    if (!c || m < 1 || m > ASP_MAX_ACTIVE || !theta || (m > 1 && !stored))
        return ASP_ERR_INVALID_ARG;
    if (m > c->opt.max_active)
        return fail(c, ASP_ERR_INVALID_ARG, "more members than the context's max_active");
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_eval_trial inside a step-API sequence");
    for (int i = 0; i < 4 * m; ++i)
        if (!isfinite(theta[i]) || (i >= 4 && !isfinite(stored[i])))
            return fail(c, ASP_ERR_INVALID_ARG, "non-finite trial parameters");
    for (int j = 0; j < m; ++j)
        if (!(theta[4 * j + 3] > 0.0) || (j > 0 && !(stored[4 * j + 3] > 0.0)))
            return fail(c, ASP_ERR_INVALID_ARG, "widths must be positive");
    const int n = 4 * m;
    const size_t nout = (size_t)asp::kMaxN * asp::kMaxN + asp::kMaxN + 3;
    if (!c->diag_out) HIP_OR_FAIL(c, dev_alloc(&c->diag_out, nout));
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    DevState *h = c->st_host;
    const int32_t stop0 = h->stop;
    h->diag_m = m;
    for (int i = 0; i < asp::kMaxN; ++i) {
        h->diag_theta[i] = i < n ? theta[i] : 0.0;
        h->diag_stored[i] = (i >= 4 && i < n) ? stored[i] : 0.0;
    }
    h->diag_out = c->diag_out;
    HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st + offsetof(DevState, diag_m), &h->diag_m,
                                  sizeof(DevState) - offsetof(DevState, diag_m),
                                  hipMemcpyHostToDevice, c->stream));
    asp::Params q = c->P;
    q.fuse_update = 0;
    HIP_OR_FAIL(c, asp::launch_fit(q, c->stream));
    std::vector<double> out((size_t)n * n + n + 3);
    HIP_OR_FAIL(c, hipMemcpyAsync(out.data(), c->diag_out, sizeof(double) * out.size(),
                                  hipMemcpyDeviceToHost, c->stream));
    s = pull_all(c);
    if (s != ASP_OK) return s;
    if (h->stop != stop0) return fail(c, ASP_ERR_DEVICE, "the evaluation's waits ran out");
    if (jtj) memcpy(jtj, out.data(), sizeof(double) * n * n);
    if (jtr) memcpy(jtr, out.data() + n * n, sizeof(double) * n);
    if (F) *F = out[n * n + n];
    if (chi2) *chi2 = out[n * n + n + 1];
    if (npx) *npx = (int64_t)out[n * n + n + 2];
    return ASP_OK;
}

asp_status asp_last_fit(asp_ctx *c, asp_fit_report *rep)
{
    if (!c || !rep) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    fill_report(c->st_host, rep);
    return ASP_OK;
}


asp_status asp_update_residual(asp_ctx *c, int64_t *pixels_touched)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->phase != 2) return fail(c, ASP_ERR_STATE, "asp_update_residual needs a fit first");
    unsigned long long px0 = 0, px1 = 0;
    asp_status s = pixels_touched ? pull_with_px(c, &px0) : ASP_OK;
    if (s != ASP_OK) return s;
    HIP_OR_FAIL(c, asp::launch_update(c->P, c->update_grid, c->stream));
    s = pull_with_px(c, &px1);
    if (s != ASP_OK) return s;
    if (pixels_touched) *pixels_touched = (int64_t)(px1 - px0);
    c->phase = 0;
    return ASP_OK;
}

asp_status asp_step(asp_ctx *c)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_step inside a step-API sequence");
    const int every = c->opt.refresh_every;
    if (every > 0) {
        asp_status r = setup_refresh(c);
        if (r != ASP_OK) return r;
    }
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    const int64_t k = c->st_host->k;
    s = enqueue_iteration(c);
    if (s != ASP_OK) return s;
    if (every > 0 && (k + 1) % every == 0) {
        s = enqueue_refresh(c, 0);
        if (s != ASP_OK) return s;
    }
    s = pull_all(c);
    if (s != ASP_OK) return s;
    s = harvest(c);
    if (s != ASP_OK) return s;
    return stop_status(c);
}

asp_status asp_run(asp_ctx *c, int64_t n_iter, asp_run_report *rep)
{
    if (!c || n_iter < 0) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_run inside a step-API sequence");
    unsigned long long up0 = 0, up1 = 0;
    asp_status s = pull_with_px(c, &up0);
    if (s != ASP_OK) return s;
    const int64_t k0 = c->st_host->k;
    const unsigned long long t0 = c->st_host->sum_trials, nc0 = c->st_host->not_converged,
                             fb0 = c->st_host->fallbacks,
                             ep0 = c->st_host->sum_eval_px, gf0 = c->st_host->sum_gram_flops,
                             sm0 = c->st_host->sum_smoothed, pk0 = c->st_host->pk_tiles_done,
                             na0 = c->st_host->not_added;
    const int every = c->opt.refresh_every;
    if (every > 0) {
        s = setup_refresh(c);
        if (s != ASP_OK) return s;
    }
    int64_t done = 0;
    asp_status result = stop_status(c);
    while (result == ASP_OK && done < n_iter) {
        const int64_t chunk = (n_iter - done) < 256 ? (n_iter - done) : 256;
        const int64_t kc = c->st_host->k;
        for (int64_t i = 0; i < chunk; ++i) {
            s = enqueue_iteration(c);
            if (s != ASP_OK) return s;
            // the exact-PSF refresh after every `every`-th iteration (a refresh
            // queued behind a stop leaves the residual alone)
            if (every > 0 && (kc + i + 1) % every == 0) {
                s = enqueue_refresh(c, 0);
                if (s != ASP_OK) return s;
            }
        }
        s = pull_all(c);
        if (s != ASP_OK) return s;
        s = harvest(c);
        if (s != ASP_OK) return s;
        const int64_t before = done;
        done = c->st_host->k - k0;
        result = stop_status(c);
        if (result == ASP_OK && done == before)
            return fail(c, ASP_ERR_STATE, "no iteration progressed and no stop was set");
    }
    s = pull_with_px(c, &up1);
    if (s != ASP_OK) return s;
    if (rep) {
        rep->iterations = c->st_host->k - k0;
        rep->total_iterations = c->st_host->k;
        rep->components = c->st_host->L;
        rep->lm_trials = (int64_t)(c->st_host->sum_trials - t0);
        rep->not_converged = (int64_t)(c->st_host->not_converged - nc0);
        rep->fallbacks = (int64_t)(c->st_host->fallbacks - fb0);
        rep->pixels_updated = (int64_t)(up1 - up0);
        rep->pixels_evaluated = (int64_t)(c->st_host->sum_eval_px - ep0);
        rep->gram_flops = (int64_t)(c->st_host->sum_gram_flops - gf0);
        rep->smoothed = (int64_t)(c->st_host->sum_smoothed - sm0);
        rep->peak_tiles_scanned = (int64_t)(c->st_host->pk_tiles_done - pk0);
        rep->not_added = (int64_t)(c->st_host->not_added - na0);
    }
    return result;
}

asp_status asp_components(asp_ctx *c, asp_component *out, int64_t cap, int64_t *n)
{
    if (!c || (!out && cap > 0) || cap < 0) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    const int64_t L = c->st_host->L;
    if (n) *n = L;
    if (!c->comp_out) HIP_OR_FAIL(c, dev_alloc(&c->comp_out, c->cap));
    const int64_t m = L < cap ? L : cap;
    if (m > 0) {
        HIP_OR_FAIL(c, asp::launch_components(c->P, c->comp_out, c->stream));
        HIP_OR_FAIL(c, hipMemcpyAsync(out, c->comp_out, sizeof(asp_component) * m,
                                      hipMemcpyDeviceToHost, c->stream));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    return cap < L ? ASP_ERR_CAPACITY : ASP_OK;
}

asp_status asp_components_raw(asp_ctx *c, double *out4, int64_t cap, int64_t *n)
{
    if (!c || (!out4 && cap > 0) || cap < 0) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    const int64_t L = c->st_host->L;
    if (n) *n = L;
    const int64_t m = L < cap ? L : cap;
    if (m > 0) {
        double *tmp = nullptr;
        HIP_OR_FAIL(c, hipHostMalloc((void **)&tmp, sizeof(double) * 4 * m, hipHostMallocDefault));
        hipError_t e = hipSuccess;
        double *src[4] = {c->ca, c->cx, c->cy, c->cs};
        for (int f = 0; f < 4 && e == hipSuccess; ++f)
            e = hipMemcpyAsync(tmp + f * m, src[f], sizeof(double) * m, hipMemcpyDeviceToHost,
                               c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            for (int64_t j = 0; j < m; ++j)
                for (int f = 0; f < 4; ++f) out4[4 * j + f] = tmp[f * m + j];
        (void)hipHostFree(tmp);
        if (e != hipSuccess) return fail(c, ASP_ERR_DEVICE, hipGetErrorString(e));
    }
    return cap < L ? ASP_ERR_CAPACITY : ASP_OK;
}

asp_status asp_residual(asp_ctx *c, float *out)
{
    if (!c || !out) return ASP_ERR_INVALID_ARG;
    HIP_OR_FAIL(c, hipMemcpyAsync(out, c->R, sizeof(float) * c->H * c->W, hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_residual_sumsq(asp_ctx *c, double *sum_sq)
{
    if (!c || !sum_sq) return ASP_ERR_INVALID_ARG;
    asp_status s = rebase_sumsq(c);
    if (s != ASP_OK) return s;
    HIP_OR_FAIL(c, hipMemcpyAsync(sum_sq, c->sumsq + 1024, sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_residual_sumsq_tracked(asp_ctx *c, double *sum_sq)
{
    if (!c || !sum_sq) return ASP_ERR_INVALID_ARG;
    HIP_OR_FAIL(c, asp::launch_sq_read(c->st, c->sumsq + 1025, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(sum_sq, c->sumsq + 1025, sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_residual_device(asp_ctx *c, float **dev)
{
    if (!c || !dev) return ASP_ERR_INVALID_ARG;
    *dev = c->R;
    return ASP_OK;
}

asp_status asp_psf_gauss(asp_ctx *c, double *alpha_b, double *omega_b)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    if (alpha_b) *alpha_b = c->st_host->alpha_b;
    if (omega_b) *omega_b = c->st_host->omega_b;
    return ASP_OK;
}

asp_status asp_fit_profile(asp_ctx *c, double *out, int32_t n)
{
    if (!c || !out || n < 0 || n > asp::kProfSlots) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    int rate_khz = 100000;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device);
    const double us_per_tick = 1000.0 / (double)(rate_khz > 0 ? rate_khz : 100000);
    for (int i = 0; i < n; ++i) {
        const double v = (double)c->st_host->prof[i];
        out[i] = (i < 9) ? v * us_per_tick : v;   // 9 timers, then counts
    }
    return ASP_OK;
}

asp_status asp_fit_histogram(asp_ctx *c, int64_t *fits, int64_t *trials, double *us, int32_t n)
{
    if (!c || n < 0 || n > ASP_MAX_ACTIVE + 1) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    int rate_khz = 100000;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device);
    const double us_per_tick = 1000.0 / (double)(rate_khz > 0 ? rate_khz : 100000);
    const DevState *h = c->st_host;
    for (int m = 0; m < n; ++m) {
        if (fits) fits[m] = (int64_t)h->fits_m[m];
        if (trials) trials[m] = (int64_t)h->trials_m[m];
        if (us) us[m] = (double)h->ticks_m[m] * us_per_tick;
    }
    return ASP_OK;
}

asp_status asp_kernel_timing(asp_ctx *c, int32_t on)
{
    if (!c || on < 0 || on > 1) return ASP_ERR_INVALID_ARG;
    if (!c->ev_kind.empty()) {
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        asp_status s = harvest(c);
        if (s != ASP_OK) return s;
    }
    c->timing = on != 0;
    for (int i = 0; i < 9; ++i) { c->t_ms[i] = 0.0; c->t_n[i] = 0; }
    return ASP_OK;
}

asp_status asp_kernel_times(asp_ctx *c, double *ms, int64_t *launches, int32_t n)
{
    if (!c || n < 0 || n > 9 || (n > 0 && (!ms || !launches))) return ASP_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i) { ms[i] = c->t_ms[i]; launches[i] = c->t_n[i]; }
    return ASP_OK;
}

asp_status asp_set_mlp(asp_ctx *c, const float *weights, int64_t n)
{
    if (!c || !weights || n != asp::kNetParams) return ASP_ERR_INVALID_ARG;
    float *flat = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&flat, sizeof(float) * asp::kNetParams));
    hipError_t e = hipMemcpyAsync(flat, weights, sizeof(float) * asp::kNetParams,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !c->net)
        e = hipMalloc(&c->net, sizeof(float) * (asp::kNetParams + asp::kNetScratch));
    if (e == hipSuccess) e = asp::launch_net_layout(flat, c->net, c->stream);
    // the proposal kernel's arrival counter starts at a multiple of its grid
    if (e == hipSuccess)
        e = hipMemsetAsync(c->net + asp::kNetParams + (int64_t)asp::kPropGroups * asp::kNetH, 0,
                           sizeof(unsigned int), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(flat);
    if (e != hipSuccess) return fail(c, ASP_ERR_DEVICE, std::string("asp_set_mlp: ") + hipGetErrorString(e));
    const int64_t n1 = (int64_t)asp::kNetH * asp::kNetIn, n2 = (int64_t)asp::kNetH * asp::kNetH;
    c->netp.w1 = c->net;
    c->netp.b1 = c->net + n1;
    c->netp.w2t = c->net + n1 + asp::kNetH;
    c->netp.b2 = c->net + n1 + asp::kNetH + n2;
    c->netp.w3 = c->net + n1 + 2 * asp::kNetH + n2;
    c->netp.b3 = c->netp.w3 + (int64_t)asp::kNetOut * asp::kNetH;
    c->netp.part = c->net + asp::kNetParams;
    c->netp.done = reinterpret_cast<unsigned int *>(c->netp.part +
                                                    (int64_t)asp::kPropGroups * asp::kNetH);
    return ASP_OK;
}

asp_status asp_set_init_mode(asp_ctx *c, int32_t mode)
{
    if (!c || mode < 0 || mode > 2) return ASP_ERR_INVALID_ARG;
    if (mode == 1 && !c->net) return fail(c, ASP_ERR_STATE, "no network set (asp_set_mlp)");
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_set_init_mode inside a step-API sequence");
    if (mode == 2) {
        if (c->in_batch)
            return fail(c, ASP_ERR_STATE, "the smoothing method is not available to batched fields");
        asp_status s = enter_smoothing(c);
        if (s != ASP_OK) return s;
    } else {
        c->P.smooth = 0;
    }
    c->opt.init_mode = mode;
    return ASP_OK;
}

asp_status asp_smooth_peak(asp_ctx *c, int32_t *scale, int64_t *idx, float *score,
                           asp_gauss *start)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->in_batch)
        return fail(c, ASP_ERR_STATE, "the smoothing method is not available to batched fields");
    asp_status s = setup_smoothing(c);
    if (s != ASP_OK) return s;
    s = timed(c, 4, [&] { return asp::launch_smooth_passes(c->P, 1, c->stream); });
    if (s == ASP_OK) s = timed(c, 5, [&] { return asp::launch_smooth_pick(c->P, 1, c->stream); });
    if (s == ASP_OK) s = pull_all(c);
    if (s == ASP_OK) s = harvest(c);
    if (s != ASP_OK) return s;
    const DevState *h = c->st_host;
    if (!h->smooth_ready) return fail(c, ASP_ERR_DEVICE, "the smoothing pick found no maximum");
    if (scale) *scale = h->smooth_scale;
    if (idx) *idx = h->smooth_idx;
    if (score) *score = h->smooth_score;
    if (start) {
        start->amp = h->smooth_start[0];
        start->x = h->smooth_start[1];
        start->y = h->smooth_start[2];
        start->width = h->smooth_start[3];
    }
    return ASP_OK;
}

asp_status asp_smooth_map(asp_ctx *c, int32_t scale, float *out)
{
    if (!c || !out) return ASP_ERR_INVALID_ARG;
    if (c->in_batch)
        return fail(c, ASP_ERR_STATE, "the smoothing method is not available to batched fields");
    asp_status s = setup_smoothing(c);
    if (s != ASP_OK) return s;
    if (scale < 0 || scale >= c->P.sm.n) return fail(c, ASP_ERR_INVALID_ARG, "no such scale");
    if (!c->sm_map) HIP_OR_FAIL(c, dev_alloc(&c->sm_map, (size_t)(c->H * c->W)));
    asp::Params P = c->P;
    P.sm.map = c->sm_map;
    P.sm.map_scale = scale;
    HIP_OR_FAIL(c, asp::launch_smooth_passes(P, 2, c->stream));
    HIP_OR_FAIL(c, asp::launch_smooth_pick(P, 2, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(out, c->sm_map, sizeof(float) * c->H * c->W,
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_refresh_residual(asp_ctx *c)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_refresh_residual inside a step-API sequence");
    asp_status s = setup_refresh(c);
    if (s == ASP_OK) s = enqueue_refresh(c, 1);
    if (s == ASP_OK) s = pull_all(c);
    if (s == ASP_OK) s = harvest(c);
    return s;
}

asp_status asp_step_2004(asp_ctx *c, asp_fit2004_report *rep)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_step_2004 inside a step-API sequence");
    if (c->in_batch)
        return fail(c, ASP_ERR_STATE, "the Asp-Clean2004 iteration is not available to batched fields");
    return step_2004(c, rep);
}

asp_status asp_set_2004_convolution(asp_ctx *c, int32_t mode)
{
    if (!c || mode < 0 || mode > 2) return ASP_ERR_INVALID_ARG;
    c->a4_conv = mode;
    return ASP_OK;
}

asp_status asp_run_2004(asp_ctx *c, int64_t n_iter, asp_run_report *rep)
{
    if (!c || n_iter < 0) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_run_2004 inside a step-API sequence");
    if (c->in_batch)
        return fail(c, ASP_ERR_STATE, "the Asp-Clean2004 iteration is not available to batched fields");
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    const DevState *h = c->st_host;
    const int64_t k0 = h->k;
    const unsigned long long t0 = h->sum_trials, nc0 = h->not_converged, ep0 = h->sum_eval_px,
                             sm0 = h->sum_smoothed, pk0 = h->pk_tiles_done;
    asp_status result = stop_status(c);
    for (int64_t i = 0; result == ASP_OK && i < n_iter; ++i) {
        s = step_2004(c, nullptr);
        if (s < 0) return s;
        result = (s == ASP_LM_NOT_CONVERGED) ? ASP_OK : s;
    }
    if (rep) {
        memset(rep, 0, sizeof *rep);
        rep->iterations = h->k - k0;
        rep->total_iterations = h->k;
        rep->components = h->L;
        rep->lm_trials = (int64_t)(h->sum_trials - t0);
        rep->not_converged = (int64_t)(h->not_converged - nc0);
        rep->pixels_evaluated = (int64_t)(h->sum_eval_px - ep0);
        rep->smoothed = (int64_t)(h->sum_smoothed - sm0);
        rep->peak_tiles_scanned = (int64_t)(h->pk_tiles_done - pk0);
    }
    return result;
}

asp_status asp_smooth_work(asp_ctx *c, int64_t *pixels, double *flops)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    int64_t px = 0;
    double fl = 0.0;
    for (int j = 0; j < c->P.sm.n; ++j) {
        const unsigned long long n = c->st_host->sm_px[j] + c->st_host->sm_px[asp::kMaxScales + j];
        px += (int64_t)n;
        fl += 2.0 * (double)(2 * c->P.sm.h[j] + 1) * (double)n;
    }
    if (pixels) *pixels = px;
    if (flops) *flops = fl;
    return ASP_OK;
}

asp_status asp_smooth_widths(asp_ctx *c, double *sigma, int32_t cap, int32_t *n)
{
    if (!c || cap < 0 || (cap > 0 && !sigma)) return ASP_ERR_INVALID_ARG;
    if (c->in_batch)
        return fail(c, ASP_ERR_STATE, "the smoothing method is not available to batched fields");
    asp_status s = setup_smoothing(c);
    if (s != ASP_OK) return s;
    const int m = c->P.sm.n;
    if (n) *n = m;
    for (int j = 0; j < m && j < cap; ++j) sigma[j] = c->P.sm.sig[j];
    return cap < m ? ASP_ERR_CAPACITY : ASP_OK;
}

asp_status asp_record(asp_ctx *c, float *patches, float *targets, int32_t *flags, int64_t cap)
{
    if (!c || cap < 0 || (cap > 0 && (!patches || !targets || !flags))) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_record inside a step-API sequence");
    c->P.rec_patch = cap > 0 ? patches : nullptr;
    c->P.rec_target = cap > 0 ? targets : nullptr;
    c->P.rec_flag = cap > 0 ? flags : nullptr;
    c->P.rec_cap = cap;
    c->st_host->rec_n = 0;
    HIP_OR_FAIL(c, hipMemcpyAsync((char *)c->st + offsetof(DevState, rec_n), &c->st_host->rec_n,
                                  sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_record_count(asp_ctx *c, int64_t *n)
{
    if (!c || !n) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    *n = c->st_host->rec_n;
    return ASP_OK;
}

asp_status asp_model_image(asp_ctx *c, float *out)
{
    if (!c || !out) return ASP_ERR_INVALID_ARG;
    if (c->in_batch) return fail(c, ASP_ERR_STATE, "the model image is not available to batched fields");
    asp_status s = setup_refresh(c);
    if (s != ASP_OK) return s;
    if (!c->model_dev) HIP_OR_FAIL(c, dev_alloc(&c->model_dev, (size_t)(c->H * c->W)));
    asp::RefreshArgs a = c->rf;
    a.force = 1;
    HIP_OR_FAIL(c, asp::render_model(a, c->model_dev, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(out, c->model_dev, sizeof(float) * c->H * c->W,
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_state_size(asp_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    *bytes = state_bytes(c->H, c->W, c->st_host->L);
    return ASP_OK;
}

asp_status asp_save_state(asp_ctx *c, void *blob, int64_t cap, int64_t *bytes)
{
    if (!c || cap < 0 || (!blob && cap > 0)) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_save_state inside a step-API sequence");
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    const DevState *h = c->st_host;
    const int64_t L = h->L, need = state_bytes(c->H, c->W, L);
    if (bytes) *bytes = need;
    if (cap < need) return fail(c, ASP_ERR_CAPACITY, "the state blob needs asp_state_size bytes");
    StateHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, kStateMagic, sizeof hd.magic);
    hd.H = c->H; hd.W = c->W; hd.k = h->k; hd.L = L;
    hd.smooth_now = h->smooth_now;
    hd.alpha_b = h->alpha_b; hd.omega_b = h->omega_b;
    char *p = (char *)blob;
    memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    HIP_OR_FAIL(c, hipMemcpyAsync(p, c->R, sizeof(float) * c->H * c->W, hipMemcpyDeviceToHost,
                                  c->stream));
    p += sizeof(float) * c->H * c->W;
    double *const lists[4] = {c->ca, c->cx, c->cy, c->cs};
    for (double *d : lists) {
        if (L) HIP_OR_FAIL(c, hipMemcpyAsync(p, d, sizeof(double) * L, hipMemcpyDeviceToHost, c->stream));
        p += sizeof(double) * L;
    }
    int64_t *const iters[2] = {c->c_added, c->c_updated};
    for (int64_t *d : iters) {
        if (L) HIP_OR_FAIL(c, hipMemcpyAsync(p, d, sizeof(int64_t) * L, hipMemcpyDeviceToHost, c->stream));
        p += sizeof(int64_t) * L;
    }
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_load_state(asp_ctx *c, const void *blob, int64_t bytes)
{
    if (!c || !blob || bytes < (int64_t)sizeof(StateHeader)) return ASP_ERR_INVALID_ARG;
    if (c->phase != 0) return fail(c, ASP_ERR_STATE, "asp_load_state inside a step-API sequence");
    if (c->in_batch) return fail(c, ASP_ERR_STATE, "a batched field cannot load a state");
    StateHeader hd;
    memcpy(&hd, blob, sizeof hd);
    if (memcmp(hd.magic, kStateMagic, sizeof hd.magic) != 0)
        return fail(c, ASP_ERR_INVALID_ARG, "not an asp state blob");
    if (hd.H != c->H || hd.W != c->W)
        return fail(c, ASP_ERR_INVALID_ARG, "the state was saved from an image of another size");
    if (hd.L < 0 || hd.k < 0 || bytes != state_bytes(hd.H, hd.W, hd.L))
        return fail(c, ASP_ERR_INVALID_ARG, "the state blob has the wrong length");
    if (hd.L > c->cap) return fail(c, ASP_ERR_CAPACITY, "the component list does not fit this context");
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    DevState *h = c->st_host;
    if (hd.alpha_b != h->alpha_b || hd.omega_b != h->omega_b)
        return fail(c, ASP_ERR_INVALID_ARG, "the state was saved with another PSF fit");
    const char *p = (const char *)blob + sizeof hd;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->R, p, sizeof(float) * c->H * c->W, hipMemcpyHostToDevice,
                                  c->stream));
    p += sizeof(float) * c->H * c->W;
    double *const lists[4] = {c->ca, c->cx, c->cy, c->cs};
    for (double *d : lists) {
        if (hd.L) HIP_OR_FAIL(c, hipMemcpyAsync(d, p, sizeof(double) * hd.L, hipMemcpyHostToDevice, c->stream));
        p += sizeof(double) * hd.L;
    }
    int64_t *const iters[2] = {c->c_added, c->c_updated};
    for (int64_t *d : iters) {
        if (hd.L) HIP_OR_FAIL(c, hipMemcpyAsync(d, p, sizeof(int64_t) * hd.L, hipMemcpyHostToDevice, c->stream));
        p += sizeof(int64_t) * hd.L;
    }
    h->k = hd.k;
    h->L = hd.L;
    h->stop = 0;                        // the loading context's options decide the next stop
    h->smooth_now = hd.smooth_now;
    h->smooth_ready = 0;
    h->fit_ready = 0;
    h->forced_idx = -1;
    h->have_proposal = 0;
    for (int i = 0; i < asp::kPeakSlots; ++i) h->peak_keys[i] = 0ull;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->st, h, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
    // the whole residual changed: every tile of the incremental searches is stale
    if (c->pk_tiles) HIP_OR_FAIL(c, asp::launch_peak_mark_all(c->P, c->stream));
    if (c->P.sm.n > 0) HIP_OR_FAIL(c, asp::launch_smooth_mark_all(c->P, c->stream));
    asp_status rs = rebase_sumsq(c);
    if (rs != ASP_OK) return rs;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return ASP_OK;
}

asp_status asp_counts(asp_ctx *c, int64_t *k, int64_t *L)
{
    if (!c) return ASP_ERR_INVALID_ARG;
    asp_status s = pull_all(c);
    if (s != ASP_OK) return s;
    if (k) *k = c->st_host->k;
    if (L) *L = c->st_host->L;
    return ASP_OK;
}

}  // extern "C"

// ===========================================================================
// Batched fields: a set of contexts run by one persistent launch (k_batch),
// captured once in a HIP graph per configuration and replayed.
// ===========================================================================

struct asp_batch {
    std::vector<asp_ctx *> ctx;
    hipStream_t stream = nullptr;
    int device = 0;
    asp::Params *d_params = nullptr;
    int32_t *d_order = nullptr;
    unsigned int *d_queue = nullptr;
    asp::FitGlobal *d_fg = nullptr;
    double *d_partials = nullptr;
    int grid = 0;
    int team = 8, solo_tiles = 8, min_tiles = 2;
    int64_t solo_peak_px = 65536, solo_update_px = 16384;
    // the captured graph and the configuration it was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t g_niter = -1;
    int g_team = 0, g_solo = 0, g_min = 0;
    std::string err;
};

namespace {

asp_status bfail(asp_batch *b, asp_status s, const std::string &msg)
{
    if (b) b->err = msg;
    return s;
}

#define BATCH_HIP(b, call)                                                            \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return bfail((b), ASP_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

void batch_release(asp_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (asp_ctx *c : b->ctx) asp_destroy(c);
    (void)hipFree(b->d_params); (void)hipFree(b->d_order); (void)hipFree(b->d_queue);
    (void)hipFree(b->d_fg); (void)hipFree(b->d_partials);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

bool team_ok(const asp_batch *b, int team)
{
    const int per_xcd = b->grid / 8;
    return team >= 1 && team <= 32 && per_xcd % team == 0;
}

// Capture the reset and the persistent launch for the current configuration.
asp_status batch_capture(asp_batch *b, int64_t n_iter)
{
    if (b->exec && b->g_niter == n_iter && b->g_team == b->team && b->g_solo == b->solo_tiles &&
        b->g_min == b->min_tiles)
        return ASP_OK;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    asp::BatchArgs a{};
    a.fields = b->d_params;
    a.order = b->d_order;
    a.queue = b->d_queue;
    a.fg = b->d_fg;
    a.partials = b->d_partials;
    a.n_iter = n_iter;
    a.solo_peak_px = b->solo_peak_px;
    a.spin_ticks = spin_limit_ticks(b->device);
    a.solo_update_px = b->solo_update_px;
    a.n_fields = (int32_t)b->ctx.size();
    a.team_size = b->team;
    a.solo_tiles = b->solo_tiles;
    a.min_tiles = b->min_tiles;
    BATCH_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = asp::launch_batch(a, b->grid, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, ASP_ERR_DEVICE, std::string("capture of the batched launch: ") +
                                            hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    BATCH_HIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_niter = n_iter;
    b->g_team = b->team;
    b->g_solo = b->solo_tiles;
    b->g_min = b->min_tiles;
    return ASP_OK;
}

}  // namespace

extern "C" {

asp_status asp_batch_create(int32_t n_fields, const float *const *dirty, const int64_t *H,
                            const int64_t *W, const float *const *psf, const int64_t *Hp,
                            const int64_t *Wp, const float *gain, const float *threshold,
                            const asp_options *opt, asp_batch **out)
{
    if (!out) return ASP_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_fields < 1 || !dirty || !H || !W || !psf || !Hp || !Wp || !gain || !threshold)
        return ASP_ERR_INVALID_ARG;
    if (opt && opt->stream) return ASP_ERR_INVALID_ARG;     // the batch owns its stream
    asp_batch *b = new (std::nothrow) asp_batch;
    if (!b) return ASP_ERR_NOMEM;
    auto bail = [&](asp_status s) { batch_release(b); delete b; return s; };
    if (hipGetDevice(&b->device) != hipSuccess) return bail(ASP_ERR_DEVICE);
    if (hipStreamCreate(&b->stream) != hipSuccess) return bail(ASP_ERR_DEVICE);
    asp_options o;
    asp_default_options(&o);
    if (opt) {
        if (opt->struct_size != (int32_t)sizeof(asp_options)) return bail(ASP_ERR_INVALID_ARG);
        o = *opt;
    }
    o.stream = b->stream;
    // the batched kernel has its own peak scan, no smoothing method and no refresh
    if (o.init_mode == 2 || o.peak_tiles || o.refresh_every) return bail(ASP_ERR_INVALID_ARG);
    for (int32_t i = 0; i < n_fields; ++i) {
        asp_ctx *c = nullptr;
        asp_status s = asp_create(dirty[i], H[i], W[i], psf[i], Hp[i], Wp[i], gain[i],
                                  threshold[i], &o, &c);
        if (s != ASP_OK) return bail(s);
        c->in_batch = true;
        b->ctx.push_back(c);
    }
    b->grid = asp::batch_grid_size(b->device);
    if (b->grid < 8) {
        fprintf(stderr, "asp_batch_create: the batched kernel's work-groups cannot all be "
                        "resident at once (private segment or no occupancy)\n");
        return bail(ASP_ERR_DEVICE);
    }
    if (!team_ok(b, b->team)) b->team = b->grid / 8;
    // the fields' parameter blocks and the order: largest first
    std::vector<asp::Params> P(n_fields);
    std::vector<int32_t> order(n_fields);
    for (int32_t i = 0; i < n_fields; ++i) { P[i] = b->ctx[i]->P; order[i] = i; }
    for (int32_t i = 1; i < n_fields; ++i)          // insertion sort, stable, by H*W descending
        for (int32_t j = i; j > 0 && H[order[j]] * W[order[j]] > H[order[j - 1]] * W[order[j - 1]]; --j)
            std::swap(order[j], order[j - 1]);
    const size_t n_rows = (size_t)2 * b->grid;        // T + groups rows per team, T <= 32
    if (dev_alloc(&b->d_params, (size_t)n_fields) != hipSuccess ||
        dev_alloc(&b->d_order, (size_t)n_fields) != hipSuccess ||
        dev_alloc(&b->d_queue, 1) != hipSuccess ||
        dev_alloc(&b->d_fg, (size_t)b->grid) != hipSuccess ||
        dev_alloc(&b->d_partials, n_rows * asp::kPartStride) != hipSuccess)
        return bail(ASP_ERR_NOMEM);
    if (hipMemcpy(b->d_params, P.data(), sizeof(asp::Params) * n_fields, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * n_fields, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_fg, 0, sizeof(asp::FitGlobal) * b->grid) != hipSuccess ||
        hipMemset(b->d_queue, 0, sizeof(unsigned int)) != hipSuccess)
        return bail(ASP_ERR_DEVICE);
    *out = b;
    return ASP_OK;
}

void asp_batch_destroy(asp_batch *b)
{
    batch_release(b);
    delete b;
}

const char *asp_batch_last_error(const asp_batch *b)
{
    return b ? b->err.c_str() : "null batch";
}

asp_status asp_batch_field(asp_batch *b, int32_t i, asp_ctx **ctx)
{
    if (!b || !ctx || i < 0 || i >= (int32_t)b->ctx.size()) return ASP_ERR_INVALID_ARG;
    *ctx = b->ctx[i];
    return ASP_OK;
}

asp_status asp_batch_config(asp_batch *b, int32_t team_size, int32_t solo_tiles,
                            int32_t min_tiles)
{
    if (!b) return ASP_ERR_INVALID_ARG;
    if (team_size != 0 && !team_ok(b, team_size))
        return bfail(b, ASP_ERR_INVALID_ARG, "team size must divide the work-groups of one XCD");
    if (solo_tiles < -1 || min_tiles < 0) return ASP_ERR_INVALID_ARG;
    if (team_size) b->team = team_size;
    if (solo_tiles) b->solo_tiles = solo_tiles < 0 ? 0 : solo_tiles;
    if (min_tiles) b->min_tiles = min_tiles;
    return ASP_OK;
}

asp_status asp_batch_get_config(asp_batch *b, int32_t *team_size, int32_t *solo_tiles,
                                int32_t *min_tiles, int32_t *grid)
{
    if (!b) return ASP_ERR_INVALID_ARG;
    if (team_size) *team_size = b->team;
    if (solo_tiles) *solo_tiles = b->solo_tiles;
    if (min_tiles) *min_tiles = b->min_tiles;
    if (grid) *grid = b->grid;
    return ASP_OK;
}

asp_status asp_batch_run(asp_batch *b, int64_t n_iter, asp_batch_report *rep)
{
    if (!b || n_iter < 0) return ASP_ERR_INVALID_ARG;
    for (asp_ctx *c : b->ctx)
        if (c->phase != 0) return bfail(b, ASP_ERR_STATE, "a field is inside a step-API sequence");
    int64_t k0 = 0;
    for (asp_ctx *c : b->ctx) {
        asp_status s = pull_all(c);
        if (s != ASP_OK) return bfail(b, s, c->err);
        k0 += c->st_host->k;
    }
    asp_status s = batch_capture(b, n_iter);
    if (s != ASP_OK) return s;
    hipEvent_t e0, e1;
    BATCH_HIP(b, hipEventCreate(&e0));
    BATCH_HIP(b, hipEventCreate(&e1));
    hipError_t e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bfail(b, ASP_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    int64_t k1 = 0, stopped = 0, errors = 0;
    for (asp_ctx *c : b->ctx) {
        s = pull_all(c);
        if (s != ASP_OK) return bfail(b, s, c->err);
        k1 += c->st_host->k;
        const int32_t st = c->st_host->stop;
        stopped += st != 0;
        errors += st < 0;
    }
    if (rep) {
        rep->iterations = k1 - k0;
        rep->fields_stopped = stopped;
        rep->fields_failed = errors;
        rep->ms = (double)ms;
    }
    return errors ? bfail(b, ASP_ERR_DEVICE, "a field failed (see its context)") : ASP_OK;
}

asp_status asp_batch_autotune(asp_batch *b, int64_t probe_iter, int32_t *team_size,
                              int32_t *solo_tiles, int32_t *min_tiles)
{
    if (!b || probe_iter < 1) return ASP_ERR_INVALID_ARG;
    // coordinate search on real chunks of the run: team size, then the solo
    // threshold, then the least tiles per work-group; each probe is scored by
    // iterations per second of its own chunk
    auto score = [&](double *ips) -> asp_status {
        asp_batch_report r{};
        asp_status s = asp_batch_run(b, probe_iter, &r);
        if (s != ASP_OK) return s;
        *ips = r.ms > 0.0 ? 1e3 * (double)r.iterations / r.ms : 0.0;
        return ASP_OK;
    };
    const int teams[] = {2, 4, 8, 16, 32};
    const int solos[] = {4, 8, 16, 32};
    const int mins[] = {1, 2, 4};
    double best = -1.0;
    int bt = b->team, bs = b->solo_tiles, bm = b->min_tiles;
    for (int t : teams) {
        if (!team_ok(b, t)) continue;
        b->team = t; b->solo_tiles = bs; b->min_tiles = bm;
        double v; asp_status s = score(&v);
        if (s != ASP_OK) return s;
        if (v > best) { best = v; bt = t; }
    }
    best = -1.0;
    for (int so : solos) {
        b->team = bt; b->solo_tiles = so; b->min_tiles = bm;
        double v; asp_status s = score(&v);
        if (s != ASP_OK) return s;
        if (v > best) { best = v; bs = so; }
    }
    best = -1.0;
    for (int mi : mins) {
        b->team = bt; b->solo_tiles = bs; b->min_tiles = mi;
        double v; asp_status s = score(&v);
        if (s != ASP_OK) return s;
        if (v > best) { best = v; bm = mi; }
    }
    b->team = bt; b->solo_tiles = bs; b->min_tiles = bm;
    if (team_size) *team_size = bt;
    if (solo_tiles) *solo_tiles = bs;
    if (min_tiles) *min_tiles = bm;
    return ASP_OK;
}

}  // extern "C"
