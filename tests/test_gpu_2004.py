"""The Asp-Clean2004 iteration on the GPU (asp_step_2004 / asp_run_2004: the
objective of Eq. 3 with the true PSF convolved in every evaluation, by FFT or
directly as two 1-D passes) against the FP64 oracle (oracle/asp2004.py).

Lockstep: before every GPU step the oracle is loaded with the GPU's residual
and component list and takes the same step.  Compared: the peak, the
smoothing start (the same scale and pixel, or a near tie within the FP32
bounds of the smoothing passes, when the oracle is given the GPU's start),
the fitted sky parameters (F to 1e-3 relative, x and y to 1e-3 max(1, s) px,
v = omega^2 to 1e-3 s^2, s = sqrt(v + omega_b^2), whenever both fits converged),
the update R_after = R_before - gain F B(*)g(theta) at the GPU's own theta
within the FP32 rounding of R plus the FP64 FFT error, and the component the
list receives."""
import math

import numpy as np
import pytest

import skygen
from oracle import asp2004 as a4
from oracle import smoothing as sm

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")

PARAM_RTOL = 1e-3


def smoothing_start_ok(g_start, g_scale, R, wb, smax):
    """The GPU's smoothing start against the oracle's score maps: the same
    (scale, pixel) or a near tie; returns True when it is the oracle's own."""
    from test_gpu_smooth import check_peak, oracle_maps
    H, W = R.shape
    idx = int(g_start[2]) * W + int(g_start[1])
    method = sm.auto_method(R.shape, wb, 5, smax)
    sc = sm.scores(R, wb, 5, smax, method=method, norm="peak")
    g = {"scale": g_scale, "idx": idx, "score": abs(sc[g_scale][3].ravel()[idx]), "start": g_start}
    return check_peak(g, R, sc, None, "start")


def errors(g, o, wb):
    s2 = o[3] + wb * wb
    s = math.sqrt(s2)
    return np.array([abs(g[0] - o[0]) / (PARAM_RTOL * max(abs(o[0]), 1e-30)),
                     abs(g[1] - o[1]) / (PARAM_RTOL * max(1.0, s)),
                     abs(g[2] - o[2]) / (PARAM_RTOL * max(1.0, s)),
                     abs(g[3] - o[3]) / (PARAM_RTOL * s2)])


def lockstep(f, steps, gain=None, need_strict=1, mode="auto", **kw):
    gain = f.gain if gain is None else gain
    ctx = asp.Context(f.dirty, f.psf, gain, f.threshold, max_iter=f.max_iter, **kw)
    ctx.set_2004_convolution(mode)
    gain = float(np.float32(gain))            # the loop gain crosses the C ABI as FP32
    ab, wb = ctx.psf_gauss()
    D = f.dirty.astype(np.float64)
    orc = a4.Oracle2004(f.dirty, f.psf, ab, wb, gain=gain, threshold=f.threshold,
                        max_iter=f.max_iter, lm_max_iter=kw.get("lm_max_iter", 100))
    n_strict = n_tie = 0
    regimes = set()
    for it in range(steps):
        R0, comps0, k0 = ctx.residual(), ctx.components_raw(), ctx.counts()[0]
        rc, rep = ctx.step_2004()
        if rc in (asp.ASP_STOP_THRESHOLD, asp.ASP_STOP_MAXITER):
            break
        if mode == "fft":
            assert rep["direct_evals"] == 0 and rep["direct_update"] == 0
        elif mode == "direct":
            assert rep["direct_evals"] == rep["evaluations"] and rep["direct_update"] == 1
        R0d = R0.astype(np.float64)
        exact = smoothing_start_ok(rep["start"], rep["scale"], R0d, wb, orc.s_max)
        orc.load_state(R0, comps0, k0)
        orep = orc.step(start=None if exact else rep["start"])
        n_tie += 0 if exact else 1
        assert rep["idx"] == orep["idx"], it
        assert np.abs(rep["theta0"] - orep["theta0"]).max() <= 1e-9 * max(1.0, abs(orep["theta0"][0]))
        assert np.allclose(rep["lo"], orep["lo"]) and np.allclose(rep["hi"], orep["hi"])
        th = rep["theta"]
        regimes.add("wide" if th[3] >= 1.0 else ("point" if th[3] == 0.0 else "narrow"))
        if rep["converged"] and orep["converged"]:
            err = errors(th, orep["theta"], wb)
            assert err.max() <= 1.0, (it, th, orep["theta"], err)
            n_strict += 1
        # the update at the GPU's own parameters
        conv = a4.Problem(R0d, f.psf, wb).convolved([gain * th[0], th[1], th[2], th[3]])
        want = R0d - conv
        got = ctx.residual().astype(np.float64)
        tol = 2.0 ** -23 * np.maximum(np.abs(R0d), np.abs(conv)) + 1e-9 * np.abs(D).max()
        assert np.all(np.abs(got - want) <= tol), (it, float((np.abs(got - want) / tol).max()))
        # the component: the convolved form of (gain F, omega)
        a_c, s_c = a4.convolved_form(gain * th[0], math.sqrt(th[3]), ab, wb)
        last = ctx.components_raw()[-1]
        assert np.allclose(last, [a_c, th[1], th[2], s_c], rtol=1e-13, atol=0.0), it
        assert ctx.counts() == (k0 + 1, comps0.shape[0] + 1)
    print(f"steps {it + 1}, strict {n_strict}, near-ties {n_tie}, regimes {sorted(regimes)}",
          flush=True)
    assert n_strict >= need_strict
    return ctx, regimes


CONVS = ["fft", "direct"]


@pytest.mark.parametrize("conv", CONVS)
def test_lockstep_evla128(conv):
    f = skygen.make_evla(128, 7, 40, 4, 10.0, 200, 1, psf_crop=128)
    ctx, regimes = lockstep(f, 8, gain=0.3, need_strict=5, mode=conv)
    ctx.close()


@pytest.mark.parametrize("conv", CONVS)
def test_lockstep_ragged_asymmetric_psf(conv):
    """A ragged image and an odd, off-centre PSF with a sidelobe: a point
    between pixels and a wide Gaussian."""
    rng = np.random.default_rng(11)
    n = 41
    pr, pc = n // 2 - 2, n // 2 + 1              # the PSF's peak pixel, off the centre
    lobes = [(1.0, 1.8, 0, 0), (0.25, 2.2, 6, -6)]     # (amplitude, width, rows, columns)
    psf = np.zeros((n, n))
    for amp, w, dr, dc in lobes:
        psf += skygen.isolated_gaussian(n, n, amp, pc + dc, pr + dr, w)
    H, W = 90, 117
    dirty = np.zeros((H, W))
    # closed forms: a point of flux 1.2 at (60.4, 30.7) and a Gaussian (F 3,
    # omega 4) at (25.2, 55.9); each PSF lobe images them at its offset
    for amp, w, dr, dc in lobes:
        dirty += skygen.isolated_gaussian(H, W, 1.2 * amp, 60.4 + dc, 30.7 + dr, w)
        s2 = 16.0 + w * w
        dirty += skygen.isolated_gaussian(H, W, 3.0 * amp * w * w / s2, 25.2 + dc, 55.9 + dr,
                                          math.sqrt(s2))
    dirty += rng.normal(0.0, 1e-3, size=(H, W))
    g = skygen.Field("ragged", dirty.astype(np.float32), psf.astype(np.float32), 0.5, 0.0, 20, 1,
                     np.zeros((0, 3)), np.zeros((0, 4)), 1e-3)
    ctx, regimes = lockstep(g, 6, need_strict=3, mode=conv)
    ctx.close()


def test_lockstep_direct_1024():
    """The direct route where the column pass takes 16-row tiles (images whose
    tiles of that height fill its grid) and the row pass several 256-column
    blocks: a 1024^2 EVLA-like field, every evaluation and update direct."""
    f = skygen.make_evla(1024, 13, 120, 6, 12.0, 50, 1, psf_crop=256)
    ctx, regimes = lockstep(f, 3, gain=0.3, need_strict=1, mode="direct")
    ctx.close()


def test_run_matches_steps_and_refresh_agrees():
    """asp_run_2004 gives the step API's state bit for bit; afterwards the
    exact-PSF refresh of the list reproduces the residual to the FP32 roundings
    of the updates."""
    f = skygen.make_evla(128, 8, 40, 4, 10.0, 200, 1, psf_crop=128)
    a = asp.Context(f.dirty, f.psf, 0.3, 0.0, max_iter=200)
    b = asp.Context(f.dirty, f.psf, 0.3, 0.0, max_iter=200)
    for _ in range(6):
        a.step_2004()
    rc, rep = b.run_2004(6)
    assert rc == asp.ASP_OK and rep["iterations"] == 6 and rep["lm_trials"] > 0
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    R = b.residual().astype(np.float64)
    b.refresh_residual()
    R2 = b.residual().astype(np.float64)
    assert np.abs(R2 - R).max() <= 8 * 2.0 ** -23 * np.abs(f.dirty).max()
    a.close()
    b.close()


def test_stops_and_refusals():
    f = skygen.make_c128(0)
    ctx = asp.Context(f.dirty, f.psf, 0.1, 10.0, max_iter=5)
    rc, rep = ctx.step_2004()
    assert rc == asp.ASP_STOP_THRESHOLD and ctx.counts() == (0, 0)
    ctx.close()
    ctx = asp.Context(f.dirty, f.psf, 0.1, 0.0, max_iter=2)
    rc, rep = ctx.run_2004(10)
    assert rc == asp.ASP_STOP_MAXITER and rep["iterations"] == 2
    ctx.close()
    ctx = asp.Context(f.dirty, f.psf, 0.1, 0.0, max_iter=10)
    ctx.find_peak()
    with pytest.raises(asp.AspError):
        ctx.step_2004()
    ctx.close()
    fields = [(g.dirty, g.psf, g.gain, g.threshold) for g in skygen.make_batch(64, 2, 50)]
    b = asp.Batch(fields)
    with pytest.raises(asp.AspError):
        b.field(0).step_2004()
    b.close()


def test_mixed_with_the_2016_iteration():
    """2016 iterations, then 2004 iterations on the same context: each side's
    update holds on the residual the other left."""
    f = skygen.make_evla(128, 9, 40, 4, 10.0, 200, 2, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, 0.2, 0.0, max_iter=200, max_active=2)
    ctx.run(20)
    ab, wb = ctx.psf_gauss()
    R0 = ctx.residual().astype(np.float64)
    rc, rep = ctx.step_2004()
    th = rep["theta"]
    g32 = float(np.float32(0.2))
    conv = a4.Problem(R0, f.psf, wb).convolved([g32 * th[0], th[1], th[2], th[3]])
    tol = 2.0 ** -23 * np.maximum(np.abs(R0), np.abs(conv)) + 1e-9 * np.abs(f.dirty).max()
    assert np.all(np.abs(ctx.residual() - (R0 - conv)) <= tol)
    rc, rep = ctx.run(5)
    assert rc == asp.ASP_OK and rep["iterations"] == 5
    ctx.close()


@pytest.mark.parametrize("mode", ["auto", "fft"])
def test_c4096_two_iterations(mode):
    """The 4096 x 4096 field: two iterations; each update against the oracle's
    FFT convolution at the GPU's parameters, at sampled pixels and in RMS."""
    f = skygen.make_c4096(4096)
    print("c4096 2004", mode, flush=True)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter)
    ctx.set_2004_convolution(mode)
    ab, wb = ctx.psf_gauss()
    D = f.dirty.astype(np.float64)
    rng = np.random.default_rng(7)
    H, W = f.shape
    for it in range(2):
        R0 = ctx.residual().astype(np.float64)
        rc, rep = ctx.step_2004()
        assert rc in (asp.ASP_OK, asp.ASP_LM_NOT_CONVERGED)
        print("  theta", rep["theta"], "trials", rep["trials"], "direct", rep["direct_evals"],
              "of", rep["evaluations"], "update", rep["direct_update"], flush=True)
        if mode == "fft":
            assert rep["direct_evals"] == 0 and rep["direct_update"] == 0
        th = rep["theta"]
        g32 = float(np.float32(f.gain))
        conv = a4.Problem(R0, f.psf, wb).convolved([g32 * th[0], th[1], th[2], th[3]])
        got = ctx.residual().astype(np.float64)
        pix = np.concatenate([[0, W - 1, (H - 1) * W, H * W - 1, rep["idx"]],
                              rng.integers(0, H * W, size=4000)])
        w = (R0 - conv).ravel()[pix]
        tol = 2.0 ** -23 * np.maximum(np.abs(R0.ravel()[pix]), np.abs(conv.ravel()[pix])) + \
            1e-9 * np.abs(D).max()
        assert np.all(np.abs(got.ravel()[pix] - w) <= tol), it
        assert abs(np.sqrt(np.mean(got ** 2)) - np.sqrt(np.mean((R0 - conv) ** 2))) <= \
            1e-6 * np.sqrt(np.mean(got ** 2))
    ctx.close()


def update_ok(ctx, R0, psf, gain, th, D):
    ab, wb = ctx.psf_gauss()
    conv = a4.Problem(R0, psf, wb).convolved([gain * th[0], th[1], th[2], th[3]])
    got = ctx.residual().astype(np.float64)
    tol = 2.0 ** -23 * np.maximum(np.abs(R0), np.abs(conv)) + 1e-9 * np.abs(D).max()
    return bool(np.all(np.abs(got - (R0 - conv)) <= tol))


def test_edge_cases():
    """Images smaller than the PSF and than the interpolation taps, a budget of
    one trial (against the oracle's), a negative source, and a full list."""
    psf = skygen.gaussian_psf(9, 2.5).astype(np.float32)
    g03 = float(np.float32(0.3))
    for shape in [(1, 1), (3, 5), (7, 1)]:
        dirty = np.zeros(shape, np.float32)
        dirty[shape[0] // 2, shape[1] // 2] = 1.0
        for conv in CONVS:
            print("shape", shape, conv, flush=True)
            ctx = asp.Context(dirty, psf, 0.3, 0.0, max_iter=5)
            ctx.set_2004_convolution(conv)
            R0 = ctx.residual().astype(np.float64)
            rc, rep = ctx.step_2004()
            assert rc in (asp.ASP_OK, asp.ASP_LM_NOT_CONVERGED), shape
            assert rep["direct_update"] == (conv == "direct"), shape
            assert update_ok(ctx, R0, psf, g03, rep["theta"], dirty), shape
            ctx.close()
    f = skygen.make_evla(128, 7, 40, 4, 10.0, 200, 1, psf_crop=128)
    g = float(np.float32(f.gain))
    ctx = asp.Context(f.dirty, f.psf, f.gain, 0.0, max_iter=5, lm_max_iter=1, smooth_norm=1)
    ab, wb = ctx.psf_gauss()
    rc, rep = ctx.step_2004()
    assert rc in (asp.ASP_OK, asp.ASP_LM_NOT_CONVERGED) and rep["trials"] == 1
    orc = a4.Oracle2004(f.dirty, f.psf, ab, wb, gain=g, lm_max_iter=1, smooth_norm="l2")
    orep = orc.step(start=rep["start"])
    assert orep["trials"] == 1 and bool(orep["converged"]) == bool(rep["converged"])
    s = math.sqrt(orep["theta"][3] + wb * wb)
    assert np.abs(rep["theta"] - orep["theta"]).max() <= 1e-6 * max(abs(orep["theta"][0]), s * s)
    ctx.close()
    # every source negative: the flux keeps the start's sign
    ctx = asp.Context(-f.dirty, f.psf, f.gain, 0.0, max_iter=5)
    R0 = ctx.residual().astype(np.float64)
    rc, rep = ctx.step_2004()
    assert rep["theta"][0] < 0.0 and rep["hi"][0] == 0.0 and rep["lo"][0] == -np.inf
    assert update_ok(ctx, R0, f.psf, g, rep["theta"], f.dirty)
    ctx.close()
    # a list of one component
    ctx = asp.Context(f.dirty, f.psf, f.gain, 0.0, max_iter=5, capacity=1)
    ctx.step_2004()
    with pytest.raises(asp.AspError):
        ctx.step_2004()
    ctx.close()


def test_convolution_mode_is_checked():
    f = skygen.make_evla(128, 7, 40, 4, 10.0, 200, 1, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, 0.0, max_iter=5)
    for bad in (-1, 3):
        with pytest.raises(asp.AspError):
            ctx.set_2004_convolution(bad)
    ctx.close()


def test_components_and_timers_after_2004_steps():
    """asp_components reads a 2004 component back as (gain F, omega) by Eqs. 5-6,
    and the kernel timers count its evaluations and updates."""
    f = skygen.make_evla(128, 7, 40, 4, 10.0, 200, 1, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, 0.0, max_iter=50)
    ctx.kernel_timing(True)
    reps = [ctx.step_2004()[1] for _ in range(3)]
    kt = ctx.kernel_times()
    assert kt["update2004"][1] == 3
    assert kt["eval2004"][1] >= sum(r["evaluations"] for r in reps)
    assert kt["eval2004"][0] > 0.0
    g = float(np.float32(f.gain))
    comps = ctx.components()
    assert len(comps) == 3
    for r, c in zip(reps, comps):
        th = r["theta"]
        assert c["flux"] == pytest.approx(g * th[0], rel=1e-12)
        assert (c["x"], c["y"]) == (th[1], th[2])
        if not c["is_point"]:
            assert c["width"] == pytest.approx(math.sqrt(th[3]), rel=1e-9)
    ctx.close()
