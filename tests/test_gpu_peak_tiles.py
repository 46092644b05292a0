"""The incremental peak search (option peak_tiles = 1) against the FP64 oracle's
peak and against the full scan: the largest |R|, the lowest row-major index on
ties (Sect. 2 step 1), from per-tile maxima that only the tiles touched by a
residual update refresh.  The answer must be the same pixel, bit for bit, so
whole runs with either search must give identical residuals."""
import numpy as np
import pytest

import oracle
import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def gauss_psf(fwhm=3.0, n=25):
    return skygen.gaussian_psf(n, fwhm).astype(np.float32)


def pair(f, **kw):
    a = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                    max_active=f.max_active, **kw)
    b = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                    max_active=f.max_active, peak_tiles=1, **kw)
    return a, b


@pytest.mark.parametrize("make,iters", [(lambda: skygen.make_c128(0), 150),
                                        (lambda: skygen.make_c1024(1000), 400)])
def test_run_matches_the_full_scan(make, iters):
    f = make()
    print("field", f.name, iters, flush=True)
    a, b = pair(f)
    ra, repa = a.run(iters)
    rb, repb = b.run(iters)
    assert (ra, repa["iterations"]) == (rb, repb["iterations"])
    assert repa["peak_tiles_scanned"] == 0
    H, W = f.shape
    ntiles = ((H + 63) // 64) * ((W + 63) // 64)
    print("tiles rescanned", repb["peak_tiles_scanned"], "of", ntiles * repb["iterations"],
          flush=True)
    assert 0 < repb["peak_tiles_scanned"] < ntiles * repb["iterations"]
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [(130, 67), (1, 1), (65, 1), (1, 200), (64, 64), (257, 129)])
def test_step_api_peak_is_the_oracle_peak(shape):
    """Every peak of a stepped run on a ragged image equals the oracle's argmax
    of the residual it was taken from."""
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    dirty = np.zeros(shape, np.float32)
    for _ in range(max(1, H * W // 300)):
        r, c = rng.integers(0, H), rng.integers(0, W)
        dirty[r, c] += rng.uniform(-1.0, 1.0)
    dirty += rng.normal(0.0, 1e-3, size=shape).astype(np.float32)
    ctx = asp.Context(dirty, gauss_psf(), 0.3, 0.0, max_iter=25, peak_tiles=1)
    for it in range(25):
        R0 = ctx.residual()
        rc, idx, val = ctx.find_peak()
        assert rc == asp.ASP_OK
        assert idx == oracle.peak(R0), (shape, it)
        assert val == R0.flat[idx]
        ctx.fit_active_set(idx)
        ctx.update_residual()
    ctx.close()


def test_ties_across_tiles():
    """Equal |values| in different tiles: the lowest row-major index, before and
    after an update elsewhere."""
    dirty = np.zeros((200, 300), np.float32)
    dirty[150, 10] = -0.5        # tile (2, 0)
    dirty[70, 250] = 0.5         # tile (1, 3): the lowest index of the three
    dirty[199, 299] = 0.5        # tile (3, 4), the ragged corner
    ctx = asp.Context(dirty, gauss_psf(), 1.0, 0.0, max_iter=10, peak_tiles=1)
    for it in range(4):
        R = ctx.residual()
        rc, idx, val = ctx.find_peak()
        assert idx == oracle.peak(R), it
        if it == 0:
            assert idx == 70 * 300 + 250
        ctx.fit_active_set(idx)
        ctx.update_residual()
    ctx.close()


def test_stop_threshold_with_tiles():
    ctx = asp.Context(np.zeros((100, 100), np.float32), gauss_psf(), 0.1, 1e-3, max_iter=10,
                      peak_tiles=1)
    rc, rep = ctx.run(10)
    assert rc == asp.ASP_STOP_THRESHOLD and rep["iterations"] == 0
    ctx.close()


def test_batch_refuses_peak_tiles():
    fields = [(f.dirty, f.psf, f.gain, f.threshold) for f in skygen.make_batch(64, 2, 50)]
    with pytest.raises(asp.AspError):
        asp.Batch(fields, peak_tiles=1)


def test_c4096_run_matches_the_full_scan():
    """The 4096 x 4096 field: 300 iterations with each search give the same
    residual and components bit for bit."""
    f = skygen.make_c4096(4096)
    print("c4096 peak tiles", flush=True)
    a, b = pair(f)
    ra, repa = a.run(300)
    rb, repb = b.run(300)
    assert ra == rb == asp.ASP_OK and repa["iterations"] == repb["iterations"] == 300
    print("tiles rescanned per iteration", repb["peak_tiles_scanned"] / 300, flush=True)
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()
