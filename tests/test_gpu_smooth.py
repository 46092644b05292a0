"""The smoothing method of initial values on the GPU (Sect. 2 step 1; Sect. 3)
against the FP64 oracle (oracle/smoothing.py and the C minor cycle).

* Smoothed images, element by element, within the FP32 error bound of the two
  1-D passes (derived below), on ragged images that span several tiles, on
  images smaller than a tile and with windows wider than the image.
* The peak over all smoothed images: the same (scale, pixel) as the oracle,
  or, where two candidates are closer than the rounding bound, one whose
  oracle score is within it; the start values from it.
* The incremental refresh after residual updates, against a full refresh and
  the oracle.
* Lockstep of the minor cycle in init mode 2 (smoothing start, active set
  around it, the 5 % switch) for both readings of the normalisation.
* The 4096 x 4096 field: widths, sampled smoothed values, the peak before and
  after device-resident iterations.
"""
import math

import numpy as np
import pytest

import oracle
import skygen
from oracle import smoothing as sm
from parity import RESID_TOL, param_errors

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")

U = 2.0 ** -24
NORM_NAMES = {0: "peak", 1: "l2"}


def fp32_bound(R, sigma, norm, method):
    """Elementwise bound of |GPU - exact| for the smoothed image of width
    sigma.  Each 1-D pass is a chain of 2h+1 FMAs (one rounding each) over
    taps rounded to FP32 (one more relative u per product), and the column
    pass is rounded to FP32 once more: |error| <= (2 (2h+1) + 4) u times the
    smoothing of |R|.  With the l2 norm the factors and their product add 4 u
    relative.  A floor of 1e-12 of the largest |R|-smoothing covers the
    oracle's own FFT rounding."""
    h = sm.halfwidth(sigma)
    Cabs, N = sm.smoothed(np.abs(R), sigma, method=method, need_norm=(norm == 1))
    b = (4 * h + 6) * U * Cabs + 1e-12 * Cabs.max()
    if norm == 1:
        b = b / np.sqrt(N) + 4 * U * Cabs / np.sqrt(N)
    return b


def make_ctx(dirty, psf, norm=0, scales=5, mode=2, **kw):
    return asp.Context(dirty, psf, 0.1, 0.0, max_iter=kw.pop("max_iter", 200),
                       max_active=kw.pop("max_active", 5), init_mode=mode, smooth_scales=scales,
                       smooth_norm=norm, **kw)


def oracle_maps(ctx, R, norm, scales, max_width=0.0, method=None):
    ab, wb = ctx.psf_gauss()
    H, W = R.shape
    smax = max(max_width if max_width > 0 else min(H, W) / 8.0, wb)
    if method is None:
        method = sm.auto_method(R.shape, wb, scales, smax)
    sc = sm.scores(R, wb, scales, smax, method=method, norm=NORM_NAMES[norm])
    return wb, smax, sc, method


def point_bound(R, sigma, p, norm):
    """fp32_bound at one pixel, by direct window sums."""
    h = sm.halfwidth(sigma)
    Cabs, N, _ = sm.score_at(np.abs(R), sigma, int(p))
    b = (4 * h + 6) * U * Cabs + 1e-12 * Cabs
    return b / math.sqrt(N) + 4 * U * Cabs / math.sqrt(N) if norm == 1 else b


def check_peak(g, R, sc, bounds, tag="", norm=0):
    """The GPU's (scale, pixel) against the oracle's score maps: a maximum
    within the rounding bound; its score and start values.  bounds: per-scale
    bound maps, or None for bounds at the two pixels involved."""
    stack = np.stack([np.abs(S).ravel() for (_, _, _, S) in sc])
    flat = int(np.argmax(stack))
    oj, op = divmod(flat, R.size)
    j, p = g["scale"], g["idx"]
    assert 0 <= j < len(sc) and 0 <= p < R.size, (tag, g)
    if bounds is None:
        bj, bo = point_bound(R, sc[j][0], p, norm), point_bound(R, sc[oj][0], op, norm)
        bo += 1e-12 * stack.max()
    else:
        bj, bo = bounds[j].ravel()[p], bounds[oj].ravel()[op]
    s_gpu = abs(sc[j][3].ravel()[p])
    tol = bj + bo
    assert s_gpu >= stack[oj, op] - tol, (tag, g, oj, op, stack[oj, op], s_gpu, tol)
    assert abs(g["score"] - s_gpu) <= bj + 1e-12 * stack.max(), (tag, g["score"], s_gpu)
    sig = sc[j][0]
    r, c = divmod(p, R.shape[1])
    C, N, _ = sm.score_at(R, sig, p)
    Cabs, _, _ = sm.score_at(np.abs(R), sig, p)
    assert abs(g["start"][0] - C / N) <= 1e-12 * Cabs / N + 1e-300, (tag, g["start"], C / N)
    assert tuple(g["start"][1:]) == (float(c), float(r), sig), (tag, g["start"])
    return (j, p) == (oj, op)


def gauss_psf(fwhm=3.06, n=33):
    return skygen.gaussian_psf(n, fwhm).astype(np.float32)


CASES = {
    # name: (image, psf, max_width, scales)
    "noise_ragged": (lambda: skygen.random_image(150, 203, 1), gauss_psf(), 0.0, 5),
    "small": (lambda: skygen.random_image(37, 50, 2), gauss_psf(), 0.0, 5),
    "field": (lambda: skygen.make_c128(3).dirty, None, 0.0, 5),
    "wide_windows": (lambda: skygen.random_image(100, 90, 3), gauss_psf(6.0, 41), 60.0, 5),
    "huge_windows": (lambda: skygen.random_image(64, 70, 4), gauss_psf(20.0, 81), 400.0, 6),
}


@pytest.mark.parametrize("norm", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_smoothed_images_and_peak(case, norm):
    make, psf, max_width, scales = CASES[case]
    img = make()
    if psf is None:
        psf = skygen.make_c128(3).psf
    print("case", case, "norm", norm, img.shape, flush=True)
    ctx = make_ctx(img, psf, norm=norm, scales=scales, max_width=max_width)
    R = ctx.residual().astype(np.float64)
    wb, smax, sc, method = oracle_maps(ctx, R, norm, scales, max_width)
    widths = ctx.smooth_widths()
    assert list(widths) == sm.widths(wb, scales, smax)
    bounds = []
    for j, (sig, C, N, S) in enumerate(sc):
        b = fp32_bound(R, sig, norm, method)
        bounds.append(b)
        got = ctx.smooth_map(j).astype(np.float64)
        err = np.abs(got - S)
        print(f"  scale {j} sigma {sig:.3f}: max err {err.max():.3e}, "
              f"max err/bound {(err / b).max():.3f}", flush=True)
        assert np.all(err <= b), (case, j, float((err / b).max()))
    g = ctx.smooth_peak()
    exact = check_peak(g, R, sc, bounds, case, norm)
    print("  peak", g["scale"], g["idx"], "same as the oracle" if exact else "near-tie", flush=True)
    ctx.close()


def test_incremental_refresh_matches_full_and_oracle():
    """Simple-method iterations update the residual while the smoothed images
    are only marked stale; the next pick refreshes the stale tiles alone."""
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=400, max_active=5,
                      smooth_scales=5)
    g0 = ctx.smooth_peak()                 # builds every tile
    for burst in range(3):
        rc, _ = ctx.run(15)                # simple values: updates mark stale tiles
        assert rc == asp.ASP_OK
        g1 = ctx.smooth_peak()             # stale tiles only
        R = ctx.residual().astype(np.float64)
        wb, smax, sc, method = oracle_maps(ctx, R, 0, 5)
        bounds = [fp32_bound(R, s, 0, method) for (s, _, _, _) in sc]
        check_peak(g1, R, sc, bounds, f"burst {burst}")
        for j, (sig, C, N, S) in enumerate(sc):
            got = ctx.smooth_map(j).astype(np.float64)   # every tile of the row pass
            assert np.all(np.abs(got - S) <= bounds[j]), (burst, j)
        g2 = ctx.smooth_peak()
        assert (g2["scale"], g2["idx"], g2["score"]) == (g1["scale"], g1["idx"], g1["score"])
        assert np.array_equal(g2["start"], g1["start"])
    assert g0["idx"] != g1["idx"] or g0["score"] != g1["score"]
    ctx.close()


def width_index(widths, s):
    j = int(np.argmin(np.abs(np.asarray(widths) - s)))
    assert widths[j] == s
    return j


def smooth_lockstep(f, norm, iters, switch_area=0, need_simple=0, need_strict=0):
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active, init_mode=2, smooth_norm=norm,
                      switch_area=switch_area)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                        max_active=f.max_active, alpha_b=ab, omega_b=wb, cap=f.max_iter + 1,
                        smooth_scales=5, smooth_norm=NORM_NAMES[norm],
                        switch_deconvolved=bool(switch_area))
    widths = list(ctx.smooth_widths())
    peak = float(np.abs(f.dirty).max())
    n_smooth = n_simple = n_strict = n_tie = 0
    prev = None
    for it in range(iters):
        R0, comps0, k0 = ctx.residual(), ctx.components_raw(), ctx.counts()[0]
        rc, idx, val = ctx.find_peak()
        if rc != 0:
            break
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        used = rep["init_source"] == 3
        if prev is not None:
            # the switch: the oracle's decision from its previous step, unless that
            # fit's area ratio sat on the 5 % boundary
            s1, s0 = prev["theta"][0, 3], prev["theta0"][0, 3]
            a1, a0 = (s1 * s1 - wb * wb, s0 * s0 - wb * wb) if switch_area else (s1 * s1, s0 * s0)
            if abs(a1 - 0.05 * a0) > 1e-6 * abs(a0):
                assert used == orc.smooth_now, it
        else:
            assert used
        orc.load_state(R0, comps0, k0)
        orc.smooth_now = used
        start = None
        if used:
            n_smooth += 1
            g_start = np.asarray(rep["init"])
            j = width_index(widths, g_start[3])
            g = {"scale": j, "idx": int(g_start[2]) * f.shape[1] + int(g_start[1]),
                 "score": None, "start": g_start}
            R64 = R0.astype(np.float64)
            _, smax, sc, method = oracle_maps(ctx, R64, norm, 5)
            g["score"] = abs(sc[j][3].ravel()[g["idx"]])     # the GPU's score is checked elsewhere
            if not check_peak(g, R64, sc, None, f"it {it}", norm):
                n_tie += 1
                start = g_start
        else:
            n_simple += 1
        orep = orc.step(start=start)
        assert orep["smoothed"] == used
        assert orep["idx"] == idx
        assert orep["members"] == rep["members"], (it, orep["members"], rep["members"])
        assert np.abs(np.asarray(rep["theta0"][0]) - orep["theta0"][0]).max() <= \
            1e-9 * max(1.0, abs(orep["theta0"][0][0])), it
        R1 = ctx.residual().astype(np.float64)
        assert np.abs(R1 - orc.R).max() <= RESID_TOL * peak, it
        if rep["converged"] and orep["converged"]:
            err = param_errors(rep["theta"], orep["theta"])
            assert err.max() <= 1.0, (it, err)
            n_strict += 1
        prev = orep
    print(f"smoothing fits {n_smooth}, simple {n_simple}, strict {n_strict}, near-ties {n_tie}",
          flush=True)
    assert n_smooth >= 1 and n_simple >= need_simple and n_strict >= need_strict
    ctx.close()


def test_lockstep_smooth_peak_norm():
    """Peak-1 beams on a 128 x 128 field: the switch fires within 60
    iterations."""
    smooth_lockstep(skygen.make_c128(0), 0, 60, need_simple=1, need_strict=40)


def test_lockstep_smooth_l2_norm():
    smooth_lockstep(skygen.make_c128(1), 1, 40, need_strict=25)


def test_lockstep_smooth_deconvolved_switch():
    smooth_lockstep(skygen.make_c128(2), 0, 40, switch_area=1, need_strict=25)


def test_run_matches_step_api_in_smoothing_mode():
    """asp_run (the device decides the switch, no host round trips) against
    the step API on the same field: identical residual and components."""
    f = skygen.make_c128(0)
    a = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=200, init_mode=2)
    b = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=200, init_mode=2)
    rc, rep = a.run(60)
    assert rc == asp.ASP_OK and rep["iterations"] == 60
    n_smooth = 0
    for it in range(60):
        rc, idx, _ = b.find_peak()
        rc, r = b.fit_active_set(idx)
        b.update_residual()
        n_smooth += r["init_source"] == 3
    assert rep["smoothed"] == n_smooth and 0 < n_smooth < 60
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (3, 5), (7, 1), (1, 9)])
def test_degenerate_shapes_smoothing_lockstep(shape):
    H, W = shape
    dirty = np.zeros(shape, np.float32)
    dirty[H // 2, W // 2] = 1.0
    if H * W > 1:
        dirty.flat[0] = -0.3
    f = skygen.Field("tiny", dirty, gauss_psf(2.5, 9), 0.3, 0.0, 6, 5, np.zeros((0, 3)),
                     np.zeros((0, 4)), 0.0)
    smooth_lockstep(f, 0, 6)


def test_threshold_stop_and_batch_refusal():
    ctx = asp.Context(np.zeros((64, 64), np.float32), gauss_psf(), 0.1, 1e-3, max_iter=10,
                      init_mode=2)
    rc, rep = ctx.run(10)
    assert rc == asp.ASP_STOP_THRESHOLD and rep["iterations"] == 0 and rep["smoothed"] == 0
    ctx.close()
    fields = [(f.dirty, f.psf, f.gain, f.threshold) for f in skygen.make_batch(64, 2, 50)]
    with pytest.raises(asp.AspError):
        asp.Batch(fields, init_mode=2)
    b = asp.Batch(fields)
    with pytest.raises(asp.AspError) as e:
        b.field(0).set_init_mode(2)
    assert e.value.status == asp.ASP_ERR_STATE
    b.close()


def test_c4096_smoothing_sampled():
    """The 4096 x 4096 field in init mode 2: trial widths, smoothed values at
    sampled pixels (edges and corners included), and the peak before and after
    80 device-resident iterations."""
    f = skygen.make_c4096(4096)
    print("c4096 smoothing", flush=True)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active, init_mode=2)
    ab, wb = ctx.psf_gauss()
    H, W = f.shape
    widths = list(ctx.smooth_widths())
    assert widths == sm.widths(wb, 5, max(min(H, W) / 8.0, wb)) and len(widths) == 5
    rng = np.random.default_rng(7)
    pix = np.concatenate([[0, W - 1, (H - 1) * W, H * W - 1, 5 * W + 4090, 4093 * W + 3],
                          rng.integers(0, H * W, size=58)])
    R = ctx.residual().astype(np.float64)
    for j, sig in enumerate(widths):
        got = ctx.smooth_map(j).ravel()
        for p in pix:
            C, N, _ = sm.score_at(R, sig, int(p))
            Cabs, _, _ = sm.score_at(np.abs(R), sig, int(p))
            assert abs(got[p] - C) <= (4 * sm.halfwidth(sig) + 6) * U * Cabs + 1e-12, (j, p)
    for phase in range(2):
        g = ctx.smooth_peak()
        R = ctx.residual().astype(np.float64)
        _, smax, sc, method = oracle_maps(ctx, R, 0, 5, method="fft")
        exact = check_peak(g, R, sc, None, f"phase {phase}")
        print("  peak", g, "exact" if exact else "near-tie", flush=True)
        del sc
        if phase == 0:
            rc, rep = ctx.run(80)
            assert rc == asp.ASP_OK and rep["smoothed"] >= 1
    ctx.close()
