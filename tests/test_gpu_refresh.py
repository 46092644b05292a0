"""The exact-PSF residual refresh on the GPU (Sect. 2 step 3,
R = I_dirty - B (*) I_model) against the FP64 oracle (oracle/refresh.py),
given the GPU's own component list.

The GPU renders and convolves in FP64 and rounds R to FP32, so the bound is
the FP32 rounding of the result plus the FP64 FFT error: |dR| <= 2^-23
max(|D|, |B (*) M|) + 1e-9 max|D| elementwise (the model's FP64 sums are
taken in another order than the oracle's)."""
import numpy as np
import pytest

import oracle
import skygen
from oracle import refresh as rf

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def check_refresh(ctx, f, tag):
    ab, wb = ctx.psf_gauss()
    comps = ctx.components_raw()
    ctx.refresh_residual()
    got = ctx.residual().astype(np.float64)
    D = f.dirty.astype(np.float64)
    want = rf.refreshed_residual(D, f.psf.astype(np.float64), comps, ab, wb)
    conv = D - want
    tol = 2.0 ** -23 * np.maximum(np.abs(D), np.abs(conv)) + 1e-9 * np.abs(D).max()
    err = np.abs(got - want)
    print(tag, "components", len(comps), "max err", err.max(), "max err/tol", (err / tol).max(),
          flush=True)
    assert np.all(err <= tol), (tag, float((err / tol).max()))
    return got, want


@pytest.mark.parametrize("iters", [0, 60])
def test_refresh_c128_gaussian_psf(iters):
    f = skygen.make_c128(0)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    if iters:
        ctx.run(iters)
    R_minor = ctx.residual().astype(np.float64)
    got, _ = check_refresh(ctx, f, f"c128 after {iters}")
    # a Gaussian PSF is its own main-lobe Gaussian: the refresh changes little.
    # What it changes comes from rendering sky components about 1 px wide
    # (interpolated below 1 px, point-sampled above): a stack of them at one
    # point source reaches 2.1e-3 of the peak here after 60 iterations.
    assert np.abs(got - R_minor).max() <= 3e-3 * np.abs(f.dirty).max()
    ctx.close()


def test_refresh_evla_field_and_a_ragged_psf():
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=400, max_active=5)
    ctx.run(150)
    check_refresh(ctx, f, "evla256 after 150")
    ctx.close()
    # a ragged image with an odd, asymmetric PSF whose peak is off its centre
    rng = np.random.default_rng(3)
    psf = skygen.gaussian_psf(31, 3.0)[2:29, 5:26].astype(np.float32)
    psf += rng.normal(0.0, 0.01, size=psf.shape).astype(np.float32)
    dirty = (rng.normal(0.0, 0.05, size=(150, 203)) +
             skygen.isolated_gaussian(150, 203, 2.0, 100.3, 70.6, 2.0)).astype(np.float32)
    g = skygen.Field("ragged", dirty, psf, 0.2, 0.0, 40, 5, np.zeros((0, 3)), np.zeros((0, 4)),
                     0.05)
    ctx = asp.Context(g.dirty, g.psf, g.gain, g.threshold, max_iter=40, max_active=5)
    ctx.run(40)
    check_refresh(ctx, g, "ragged after 40")
    ctx.close()


def test_periodic_refresh_in_run():
    """refresh_every = 50: after each 50 iterations of asp_run the residual is
    the exact one of the component list at that point."""
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=400, max_active=5,
                      refresh_every=50)
    ab, wb = ctx.psf_gauss()
    D = f.dirty.astype(np.float64)
    for block in range(3):
        rc, rep = ctx.run(50)
        assert rc == asp.ASP_OK and rep["iterations"] == 50
        got = ctx.residual().astype(np.float64)
        want = rf.refreshed_residual(D, f.psf.astype(np.float64), ctx.components_raw(), ab, wb)
        tol = 2.0 ** -23 * np.maximum(np.abs(D), np.abs(D - want)) + 1e-9 * np.abs(D).max()
        assert np.all(np.abs(got - want) <= tol), block
    kt = ctx.kernel_times()
    ctx.close()


def test_refresh_keeps_the_incremental_searches_consistent():
    """After a refresh every tile of the incremental peak search and of the
    smoothed images is stale: the next peaks are the oracle's."""
    from oracle import smoothing as sm
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=400, max_active=5,
                      peak_tiles=1, smooth_scales=5)
    ctx.smooth_peak()
    ctx.run(100)
    ctx.refresh_residual()
    R = ctx.residual()
    rc, idx, val = ctx.find_peak()
    assert idx == oracle.peak(R)
    g = ctx.smooth_peak()
    ab, wb = ctx.psf_gauss()
    b = sm.best(R.astype(np.float64), wb, 5, max(256 / 8.0, wb), method="fft")
    if (g["scale"], g["idx"]) != (b["scale"], b["idx"]):
        # a near tie within the FP32 rounding of the two passes
        assert abs(g["score"] - abs(b["score"])) <= 1e-4 * abs(b["score"])
    ctx.close()


def test_refresh_on_degenerate_shapes_and_batch_refusal():
    for shape in [(1, 1), (3, 5), (7, 1)]:
        dirty = np.zeros(shape, np.float32)
        dirty[shape[0] // 2, shape[1] // 2] = 1.0
        psf = skygen.gaussian_psf(9, 2.5).astype(np.float32)
        g = skygen.Field("tiny", dirty, psf, 0.3, 0.0, 5, 5, np.zeros((0, 3)), np.zeros((0, 4)), 0.0)
        ctx = asp.Context(g.dirty, g.psf, g.gain, g.threshold, max_iter=5)
        ctx.run(5)
        check_refresh(ctx, g, f"tiny {shape}")
        ctx.close()
    fields = [(f.dirty, f.psf, f.gain, f.threshold) for f in skygen.make_batch(64, 2, 50)]
    with pytest.raises(asp.AspError):
        asp.Batch(fields, refresh_every=10)


def test_refresh_c4096_sampled():
    """The 4096 x 4096 field after 100 iterations: the refreshed residual
    against the oracle's FFT refresh at sampled pixels (edges and corners
    included) and in its RMS."""
    f = skygen.make_c4096(4096)
    print("c4096 refresh", flush=True)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    ctx.run(100)
    ab, wb = ctx.psf_gauss()
    comps = ctx.components_raw()
    ctx.refresh_residual()
    got = ctx.residual().astype(np.float64)
    D = f.dirty.astype(np.float64)
    want = rf.refreshed_residual(D, f.psf.astype(np.float64), comps, ab, wb)
    H, W = f.shape
    rng = np.random.default_rng(5)
    pix = np.concatenate([[0, W - 1, (H - 1) * W, H * W - 1], rng.integers(0, H * W, size=4000)])
    g, w, d = got.ravel()[pix], want.ravel()[pix], D.ravel()[pix]
    tol = 2.0 ** -23 * np.maximum(np.abs(d), np.abs(d - w)) + 1e-9 * np.abs(D).max()
    assert np.all(np.abs(g - w) <= tol)
    assert abs(np.sqrt(np.mean(got ** 2)) - np.sqrt(np.mean(want ** 2))) <= 1e-6 * np.sqrt(np.mean(want ** 2))
    ctx.close()
