"""Pins of the exact-PSF refresh oracle (oracle/refresh.py), Sect. 2 step 3:
R = I_dirty - B (*) I_model.  The checks come from outside the oracle: a
delta model against a shifted PSF written out by hand (orientation and
centring), closed forms of Gaussians convolved with a Gaussian PSF, the
band-limited shift of a point between pixels, flux and centroid of the
interpolated components, and linearity."""
import math

import numpy as np
import pytest

import skygen
from oracle import refresh as rf


def comp_for(F, omega, x, y, alpha_b, omega_b):
    """The convolved-space (a, x, y, s) whose Eq. 5-6 deconvolution is
    (F, omega) -- the forward direction written out."""
    s = math.sqrt(omega * omega + omega_b * omega_b)
    a = F * alpha_b * omega_b * omega_b / (s * s)
    return [a, x, y, s]


def test_delta_model_is_the_shifted_psf():
    """A point on a pixel contributes F B(ci + r - r0, cj + c - c0): checked with
    an asymmetric random PSF whose peak is off its centre."""
    rng = np.random.default_rng(1)
    psf = rng.uniform(-0.2, 0.5, size=(9, 13))
    psf[3, 8] = 1.0                               # the peak pixel (ci, cj) = (3, 8)
    H, W = 20, 24
    ob = 1.3
    r0, c0, F = 11, 7, 2.5
    comps = np.array([comp_for(F, 0.0, c0, r0, 1.0, ob)])
    M = rf.model_image((H, W), comps, 1.0, ob)
    assert M[r0, c0] == pytest.approx(F, rel=1e-12) and np.abs(M).sum() == pytest.approx(F)
    conv = rf.convolve_psf(M, psf)
    want = np.zeros((H, W))
    for r in range(H):
        for c in range(W):
            pr, pc = 3 + r - r0, 8 + c - c0
            if 0 <= pr < 9 and 0 <= pc < 13:
                want[r, c] = F * psf[pr, pc]
    assert np.abs(conv - want).max() <= 1e-12


def test_gaussian_psf_closure_matches_the_convolved_components():
    """With an exact Gaussian PSF, B (*) (component) is the component's own
    convolved Gaussian (a, s): the refresh of a component list equals the
    dirty image minus those Gaussians, as the minor cycle subtracts them."""
    fwhm = 4.0
    n = 41
    psf = skygen.gaussian_psf(n, fwhm)
    ob = fwhm / skygen.FWHM_PER_SIGMA
    H, W = 96, 80
    comps = np.array([comp_for(3.0, 2.5, 30.0, 40.0, 1.0, ob),
                      comp_for(-1.2, 5.0, 55.3, 47.8, 1.0, ob),
                      comp_for(0.7, 1.5, 20.6, 70.2, 1.0, ob)])
    M = rf.model_image((H, W), comps, 1.0, ob)
    conv = rf.convolve_psf(M, psf)
    want = np.zeros((H, W))
    for a, x, y, s in comps:
        want += skygen.isolated_gaussian(H, W, a, x, y, s)
    assert np.abs(conv - want).max() <= 1e-5 * np.abs(want).max()


@pytest.mark.parametrize("fx,fy", [(0.5, 0.0), (0.25, 0.75), (0.9, 0.3)])
def test_point_between_pixels_moves_the_psf(fx, fy):
    """A point at a sub-pixel position with a smooth (band-limited to double
    precision) Gaussian PSF of sigma 3 px: B (*) M is the PSF centred on the
    point, to the accuracy of the Lanczos-3 interpolation."""
    sig = 3.0
    n = 49
    psf = skygen.gaussian_psf(n, sig * skygen.FWHM_PER_SIGMA)
    H = W = 64
    x, y = 30 + fx, 28 + fy
    comps = np.array([comp_for(1.0, 0.0, x, y, 1.0, sig)])
    M = rf.model_image((H, W), comps, 1.0, sig)
    assert M.sum() == pytest.approx(1.0, rel=1e-12)
    # Lanczos-3 keeps the first moment to about 0.02 px (exactly at half pixels)
    rr, cc = np.mgrid[0:H, 0:W]
    assert (M * cc).sum() == pytest.approx(x, abs=0.025)
    assert (M * rr).sum() == pytest.approx(y, abs=0.025)
    conv = rf.convolve_psf(M, psf)
    want = skygen.isolated_gaussian(H, W, 1.0, x, y, sig)
    err = np.abs(conv - want).max()
    print("sub-pixel point, max error", err)
    assert err <= 5e-3
    # against the whole-pixel placement the interpolation is far better
    Mr = np.zeros((H, W))
    Mr[int(round(y)), int(round(x))] = 1.0
    assert err <= 0.25 * np.abs(rf.convolve_psf(Mr, psf) - want).max()


@pytest.mark.parametrize("omega", [0.3, 0.7, 0.99])
def test_narrow_component_flux_and_centroid(omega):
    H = W = 40
    x, y, F = 17.37, 21.81, 2.0
    ob = 1.5
    comps = np.array([comp_for(F, omega, x, y, 1.0, ob)])
    M = rf.model_image((H, W), comps, 1.0, ob)
    rr, cc = np.mgrid[0:H, 0:W]
    assert M.sum() == pytest.approx(F, rel=1e-12)
    assert (M * cc).sum() / F == pytest.approx(x, abs=0.025)
    assert (M * rr).sum() / F == pytest.approx(y, abs=0.025)


def test_wide_component_is_sampled_with_its_flux():
    H = W = 90
    ob = 1.5
    comps = np.array([comp_for(4.0, 6.0, 44.2, 40.7, 1.0, ob)])
    M = rf.model_image((H, W), comps, 1.0, ob)
    assert M.sum() == pytest.approx(4.0, rel=1e-6)            # the sampled Gaussian's sum
    want = skygen.isolated_gaussian(H, W, 4.0 / (2 * math.pi * 36.0), 44.2, 40.7, 6.0)
    h = 30                                        # max(3, ceil(5 omega)) around the rounded centre
    win = np.zeros((H, W), bool)
    win[41 - h:41 + h + 1, 44 - h:44 + h + 1] = True
    assert np.abs(M - want)[win].max() <= 1e-15
    assert np.all(M[~win] == 0.0)


def test_refresh_is_linear_and_empty_model_keeps_the_dirty_image():
    rng = np.random.default_rng(4)
    psf = skygen.gaussian_psf(21, 3.5)
    dirty = rng.normal(size=(50, 60))
    ob = 3.5 / skygen.FWHM_PER_SIGMA
    A = np.array([comp_for(1.0, 0.0, 10.4, 20.2, 1.0, ob), comp_for(2.0, 3.0, 30.0, 25.5, 1.0, ob)])
    B = np.array([comp_for(-0.5, 0.5, 40.9, 10.1, 1.0, ob)])
    rA = rf.refreshed_residual(dirty, psf, A, 1.0, ob)
    rB = rf.refreshed_residual(dirty, psf, B, 1.0, ob)
    rAB = rf.refreshed_residual(dirty, psf, np.vstack([A, B]), 1.0, ob)
    assert np.abs((rA + rB - dirty) - rAB).max() <= 1e-12
    assert np.array_equal(rf.refreshed_residual(dirty, psf, np.zeros((0, 4)), 1.0, ob), dirty)
