"""The residual update at the end of the fit kernel (asp_run's default) against
its own launch (update_launch=1, as asp_update_residual runs it): every pixel
is rewritten by one work-group with the same arithmetic in the same order, so
the two runs must agree bit for bit, including the stale-tile marking of the
incremental peak search and of the smoothed images."""
import numpy as np
import pytest

import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def make(f, **kw):
    opts = {"max_iter": 400, "max_active": f.max_active}
    opts.update(kw)
    return asp.Context(f.dirty, f.psf, f.gain, f.threshold, **opts)


@pytest.mark.parametrize("kw", [{}, {"init_mode": 2, "peak_tiles": 1}, {"refresh_every": 20}],
                         ids=["simple", "smoothing+tiles", "refresh"])
def test_fused_update_equals_its_own_launch(kw):
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    a = make(f, update_launch=0, **kw)
    b = make(f, update_launch=1, **kw)
    a.kernel_timing(True)
    b.kernel_timing(True)
    ra = a.run(120)
    rb = b.run(120)
    assert ra == rb
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    ka, kb = a.kernel_times(), b.kernel_times()
    assert ka["update"][1] == 0 and kb["update"][1] == 120
    # the tracked sum of R^2 follows both (the slots differ, the sum agrees)
    for c in (a, b):
        want = float(np.sum(c.residual().astype(np.float64) ** 2))
        assert abs(c.residual_sumsq(tracked=True) - want) <= 1e-12 * float(
            np.sum(f.dirty.astype(np.float64) ** 2))
    a.close()
    b.close()


def test_fused_update_c4096():
    f = skygen.make_c4096(4096)
    a = make(f, update_launch=0)
    b = make(f, update_launch=1)
    ra = a.run(60)
    rb = b.run(60)
    assert ra == rb
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()


def test_update_launch_option_is_checked():
    f = skygen.make_c128(0)
    with pytest.raises(asp.AspError):
        make(f, update_launch=2)
    with pytest.raises(asp.AspError):
        make(f, reserved=1)


def test_fused_update_on_windows_of_millions_of_pixels():
    """One extended Gaussian (sigma 150 px) on a 2048^2 field: every update
    rewrites more than 1024^2 pixels, so each work-group of both paths (256
    in the fit kernel, 4 per CU in its own launch) takes several tiles."""
    n, sig = 2048, 150.0
    y = np.arange(n, dtype=np.float64)[:, None] - n / 2.0
    x = np.arange(n, dtype=np.float64)[None, :] - n / 2.0
    dirty = np.exp(-(x * x + y * y) / (2.0 * sig * sig)).astype(np.float32)
    psf = skygen.gaussian_psf(33, 3.0).astype(np.float32)
    ctxs = [asp.Context(dirty, psf, 0.1, 0.0, max_iter=10, max_active=1, update_launch=u)
            for u in (0, 1)]
    reps = [c.run(5) for c in ctxs]
    assert reps[0] == reps[1]
    assert reps[0][1]["pixels_updated"] > 5 * 1024 * 1024
    a, b = ctxs
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    # the step API's count of one more update equals the run's
    rc, idx, _ = b.find_peak()
    b.fit_active_set(idx)
    px = b.update_residual()
    rc, r = a.run(1)
    assert r["pixels_updated"] == px > 1024 * 1024
    assert np.array_equal(a.residual(), b.residual())
    for c in ctxs:
        c.close()
