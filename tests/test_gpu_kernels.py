"""Kernel-level parity on the GPU through the C ABI: peak search, the PSF
main-lobe fit, residual updates at the image edges, the component output."""
import math

import numpy as np
import pytest

import oracle
import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def psf_small():
    return skygen.gaussian_psf(33, 3.0).astype(np.float32)


def peak_of(img):
    ctx = asp.Context(img, psf_small(), 0.1, 0.0, max_iter=10)
    rc, idx, val = ctx.find_peak()
    ctx.close()
    return rc, idx, val


CASES = [
    ("random", lambda: skygen.random_image(64, 64, 1)),
    ("odd", lambda: skygen.random_image(37, 53, 2)),
    ("tail3", lambda: skygen.random_image(1, 7, 3)),
    ("single", lambda: np.array([[-2.5]], np.float32)),
    ("all_ties", lambda: np.full((19, 23), 0.5, np.float32)),
    ("ints", lambda: skygen.random_image(128, 96, 4, "int")),
    ("zeros", lambda: np.zeros((16, 16), np.float32)),
    ("neg_peak", lambda: (lambda a: (a.__setitem__((40, 3), -9.0), a)[1])(skygen.random_image(64, 64, 5))),
    ("signed_zero", lambda: np.array([[-0.0, 0.0], [0.0, -0.0]], np.float32)),
    ("big_ragged", lambda: skygen.random_image(1023, 1027, 6, "int")),
    ("c4096_shape", lambda: skygen.random_image(4096, 4096, 7, "int")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_peak_bit_exact(name, make):
    img = np.ascontiguousarray(make(), dtype=np.float32)
    print("case", name, img.shape, flush=True)
    rc, idx, val = peak_of(img)
    assert rc == asp.ASP_OK
    assert idx == oracle.peak(img.astype(np.float64))
    assert val == img.ravel()[idx]


def test_peak_tie_at_first_index_large():
    img = np.zeros((2048, 2048), np.float32)
    for r, c in [(2047, 2047), (1500, 3), (700, 2000), (700, 1999)]:
        img[r, c] = -3.0
    rc, idx, val = peak_of(img)
    assert idx == 700 * 2048 + 1999 and val == -3.0


@pytest.mark.parametrize("fwhm", [2.5, 3.0, 4.7, 6.0])
def test_psf_fit_matches_oracle(fwhm):
    psf = skygen.gaussian_psf(64, fwhm).astype(np.float32)
    ctx = asp.Context(np.ones((8, 8), np.float32), psf, 0.1, 0.0)
    ab, wb = ctx.psf_gauss()
    ctx.close()
    oa, ow, _ = oracle.psf_fit(psf.astype(np.float64))
    assert ab == pytest.approx(oa, rel=1e-10) and wb == pytest.approx(ow, rel=1e-10)
    assert wb == pytest.approx(fwhm / skygen.FWHM_PER_SIGMA, rel=1e-6)


def test_psf_fit_yarray_matches_oracle():
    g = skygen.yarray_uv_grid(512)
    psf = np.fft.fftshift(skygen.psf_from_grid(g))[256 - 64:256 + 64, 256 - 64:256 + 64]
    psf = psf.astype(np.float32)
    ctx = asp.Context(np.ones((8, 8), np.float32), psf, 0.1, 0.0)
    ab, wb = ctx.psf_gauss()
    ctx.close()
    oa, ow, _ = oracle.psf_fit(psf.astype(np.float64))
    assert ab == pytest.approx(oa, rel=1e-10) and wb == pytest.approx(ow, rel=1e-10)


@pytest.mark.parametrize("where", ["top_left", "top_right", "bottom_left", "bottom_right"])
def test_update_windows_clipped_at_edges(where):
    H, W = 48, 40
    r, c = {"top_left": (1, 2), "top_right": (0, 38), "bottom_left": (46, 0),
            "bottom_right": (47, 39)}[where]
    img = skygen.isolated_gaussian(H, W, 1.0, c + 0.3, r - 0.2, 2.2).astype(np.float32)
    ctx = asp.Context(img, psf_small(), 0.5, 0.0, max_iter=5, max_active=3)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(img, gain=0.5, max_iter=5, max_active=3, alpha_b=ab, omega_b=wb)
    for _ in range(3):
        R0, c0 = ctx.residual(), ctx.components_raw()
        k0, _ = ctx.counts()
        assert ctx.step() == asp.ASP_OK
        orc.load_state(R0, c0, k0)
        orep = orc.step()
        assert np.abs(ctx.residual().astype(np.float64) - orc.R).max() <= 1e-4 * img.max()
        g = ctx.components_raw()
        np.testing.assert_allclose(g[-1, [0, 3]], [0.5 * orep["theta"][0, 0], orep["theta"][0, 3]],
                                   rtol=1e-3)
        np.testing.assert_allclose(g[-1, 1:3], orep["theta"][0, 1:3], atol=1e-3 * 2.2)


def test_components_eq56():
    f = skygen.make_c128(0)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    ctx.run(60)
    ab, wb = ctx.psf_gauss()
    comps = ctx.components()
    raw = ctx.components_raw()
    assert len(comps) == len(raw) == 60
    for c, (a, x, y, s) in zip(comps, raw):
        flux, alpha, omega, is_point = oracle.deconvolve(a, s, ab, wb)
        assert c["flux"] == pytest.approx(flux, rel=1e-12)
        assert c["width"] == pytest.approx(omega, rel=1e-12, abs=1e-12)
        assert bool(c["is_point"]) == is_point
        assert c["amp"] == pytest.approx(alpha, rel=1e-12)
        assert (c["x"], c["y"], c["amp_c"], c["width_c"]) == (x, y, a, s)
    assert list(comps["iter_added"]) == list(range(60))
    ctx.close()
