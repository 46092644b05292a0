"""Pins of the Asp-Clean2004 oracle (oracle/asp2004.py): the LM fit of Eq. 3,
chi^2 = || R - B (*) g(theta) ||^2, with the true PSF convolved in every
evaluation.  The checks come from outside the oracle: central finite
differences of the rendered images, the closed form of a Gaussian sky
component convolved with a Gaussian PSF (alone and with an offset sidelobe,
which fixes the orientation of the convolution), the shifted PSF of a point
between pixels, and the exact-PSF refresh oracle for the residual update.  The
rendered images are also checked to be sums of outer products of per-axis
factors, the structure both GPU convolutions (separable spectra and the
two-pass direct sum) are built on."""
import math

import numpy as np
import pytest

import skygen
from oracle import asp2004 as a4
from oracle import refresh as rf


def closed_form(H, W, F, omega, x, y, lobes):
    """B (*) sky for a sky Gaussian of flux F and width omega and a PSF that is a
    sum of Gaussians (amplitude, width, row offset, column offset): each lobe
    gives F amp w^2 / (omega^2 + w^2) exp(-|p - c - off|^2 / (2 (omega^2 + w^2)))."""
    out = np.zeros((H, W))
    for amp, w, dr, dc in lobes:
        s2 = omega * omega + w * w
        out += skygen.isolated_gaussian(H, W, F * amp * w * w / s2, x + dc, y + dr, math.sqrt(s2))
    return out


def psf_of(lobes, n=65):
    c = n // 2
    psf = np.zeros((n, n))
    for amp, w, dr, dc in lobes:
        psf += skygen.isolated_gaussian(n, n, amp, c + dc, c + dr, w)
    return psf


@pytest.mark.parametrize("x,y,v", [(10.3, 12.7, 2.3 ** 2), (15.37, 14.81, 0.45 ** 2),
                                   (9.62, 20.18, 0.0), (20.5, 11.25, 0.93 ** 2),
                                   (14.2, 16.6, 2e-4 ** 2)])
def test_derivatives_against_finite_differences(x, y, v):
    """dg/dx, dg/dy, dg/dv (v = omega^2) against central differences, one-sided
    at the bound v = 0 (where the rendering is smooth in v, not in omega)."""
    shape = (32, 36)
    g, gx, gy, gv = a4.unit_images(shape, x, y, v)
    for k, d in enumerate((gx, gy, gv)):
        if k == 2 and v < 1e-6:
            h = 1e-9
            fd = (a4.unit_images(shape, x, y, v + h)[0] - g) / h
            assert np.abs(d).max() > 1e-2          # not zero at a point source
            assert np.abs(fd - d).max() <= 1e-5 * max(1.0, np.abs(d).max()), k
            continue
        h = 1e-6 if k < 2 else 1e-6 * max(v, 1e-3)
        e = np.zeros(3)
        e[k] = h
        gp = a4.unit_images(shape, x + e[0], y + e[1], v + e[2])[0]
        gm = a4.unit_images(shape, x - e[0], y - e[1], v - e[2])[0]
        fd = (gp - gm) / (2 * h)
        assert np.abs(fd - d).max() <= 1e-6 * max(1.0, np.abs(d).max()), k


def _rank(m, rel=1e-12):
    sv = np.linalg.svd(m, compute_uv=False)
    return int(np.sum(sv > rel * sv[0])) if sv[0] > 0 else 0


@pytest.mark.parametrize("x,y,v", [(10.3, 12.7, 2.3 ** 2), (15.37, 14.81, 0.45 ** 2),
                                   (9.62, 20.18, 0.0), (1.2, 30.6, 3.1 ** 2),
                                   (0.4, 0.3, 0.2 ** 2), (34.8, 2.2, 6.5 ** 2)])
def test_rendering_is_a_sum_of_outer_products(x, y, v):
    """The structure the GPU's convolutions rely on: g = a0 b0^T, dg/dx = a0 b1^T,
    dg/dy = a1 b0^T and dg/dv = a2 b0^T + a0 b2^T, for sampled and interpolated
    components, clipped at the image's edges or not.  Checked by ranks: g, dg/dx
    and dg/dy have rank 1; g beside dg/dx (the same row factor) and g above
    dg/dy (the same column factor) too; dg/dv has rank 2 and shares a0 and b0."""
    shape = (32, 36)
    g, gx, gy, gv = a4.unit_images(shape, x, y, v)
    assert _rank(g) == 1 and _rank(gx) == 1 and _rank(gy) == 1
    assert _rank(np.hstack([g, gx])) == 1 and _rank(np.vstack([g, gy])) == 1
    assert _rank(gv) <= 2
    assert _rank(np.hstack([g, gv])) <= 2 and _rank(np.vstack([g, gv])) <= 2
    # and not trivially: a non-separable image fails the same test
    q = g + np.roll(g, 3, axis=0) * np.roll(g, 2, axis=1) / max(g.max(), 1e-300)
    assert _rank(q) > 1


def test_unit_flux():
    # narrow: the per-axis weights are normalised
    assert a4.unit_images((40, 40), 17.3, 20.6, 0.6)[0].sum() == pytest.approx(1.0, abs=1e-14)
    # wide: the sampled Gaussian of unit flux less its tail outside 5 omega
    assert a4.unit_images((60, 60), 30.2, 28.9, 2.3)[0].sum() == pytest.approx(1.0, abs=2e-6)


def test_start_conversion_round_trip():
    ab, wb = 0.9, 1.7
    for s in (wb, 2 * wb, 4 * wb):
        th = a4.start_from_smoothing([0.37, 11.0, 13.0, s], ab, wb)
        assert th[3] == pytest.approx(s * s - wb * wb, abs=1e-14)
        a, s2 = a4.convolved_form(th[0], math.sqrt(th[3]), ab, wb)
        assert a == pytest.approx(0.37, rel=1e-14) and s2 == pytest.approx(s, rel=1e-14)
    assert a4.start_from_smoothing([1.0, 0, 0, wb], ab, wb)[3] == 0.0


def run_one(dirty, psf, wb, ab=1.0, **kw):
    o = a4.Oracle2004(dirty, psf, ab, wb, gain=1.0, smooth_scales=4, **kw)
    return o, o.step()


def test_gaussian_psf_recovers_the_sky_component():
    """An exact Gaussian PSF: the fit reaches the closed form's parameters."""
    wb = 4.0 / skygen.FWHM_PER_SIGMA
    lobes = [(1.0, wb, 0, 0)]
    H, W = 64, 72
    F, om, x, y = 3.0, 2.5, 30.3, 33.6
    D = closed_form(H, W, F, om, x, y, lobes)
    o, rep = run_one(D, psf_of(lobes), wb)
    assert rep["converged"]
    th = rep["theta"]
    assert th[0] == pytest.approx(F, rel=2e-4)
    assert math.sqrt(th[3]) == pytest.approx(om, rel=2e-4)
    assert th[1] == pytest.approx(x, abs=2e-4) and th[2] == pytest.approx(y, abs=2e-4)
    assert rep["chi2_final"] <= 1e-8 * rep["chi2_init"]
    # F(theta) is chi^2 less the constant sum of R^2
    prob = a4.Problem(D, psf_of(lobes), wb)
    obj, chi2, _, _ = prob.evaluate(th, want_jac=False)
    assert obj + float(np.sum(D * D)) == pytest.approx(chi2, rel=1e-9, abs=1e-12 * np.sum(D * D))


def test_asymmetric_psf_fixes_the_orientation():
    """A PSF with a sidelobe 6 rows down and 4 columns left of its peak: B (*) sky
    carries the sidelobe image at (x - 4, y + 6).  Only the convolution (not the
    correlation) reaches chi^2 ~ 0."""
    wb = 1.7
    lobes = [(1.0, wb, 0, 0), (0.3, 2.0, 6, -4)]
    H, W = 72, 80
    F, om, x, y = 2.0, 2.0, 28.4, 30.7
    D = closed_form(H, W, F, om, x, y, lobes)
    psf = psf_of(lobes)
    o, rep = run_one(D, psf, wb)
    th = rep["theta"]
    assert rep["chi2_final"] <= 1e-8 * rep["chi2_init"]
    assert th[0] == pytest.approx(F, rel=2e-4) and math.sqrt(th[3]) == pytest.approx(om, rel=2e-4)
    assert th[1] == pytest.approx(x, abs=2e-4) and th[2] == pytest.approx(y, abs=2e-4)
    # the residual after the (gain 1) update is the closed form's leftover
    assert np.abs(o.R).max() <= 1e-4 * np.abs(D).max()
    # the mirrored sidelobe does not fit
    Dm = closed_form(H, W, F, om, x, y, [(1.0, wb, 0, 0), (0.3, 2.0, -6, 4)])
    o2, rep2 = run_one(Dm, psf, wb)
    assert rep2["chi2_final"] >= 1e-3 * rep2["chi2_init"]


@pytest.mark.parametrize("fx,fy", [(0.5, 0.25), (0.2, 0.7)])
def test_point_between_pixels(fx, fy):
    """A point of flux 1.5 at a sub-pixel position under a smooth Gaussian PSF of
    width 2 px: the fitted point (narrow rendering) lands on it to the accuracy
    of the Lanczos-3 interpolation."""
    wb = 2.0
    lobes = [(1.0, wb, 0, 0)]
    H = W = 48
    x, y = 22 + fx, 24 + fy
    D = 1.5 * skygen.isolated_gaussian(H, W, 1.0, x, y, wb)
    o, rep = run_one(D, psf_of(lobes), wb)
    th = rep["theta"]
    assert th[3] <= 0.35 ** 2
    assert th[0] == pytest.approx(1.5, rel=2e-2)
    assert th[1] == pytest.approx(x, abs=0.03) and th[2] == pytest.approx(y, abs=0.03)
    assert rep["chi2_final"] <= 1e-3 * rep["chi2_init"]


def test_update_is_the_exact_residual_of_the_list():
    """After several iterations on a field with an interferometric PSF, the
    residual is I_dirty - B (*) I_model of the component list as the exact-PSF
    refresh oracle renders it."""
    f = skygen.make_evla(64, 21, 8, 2, 6.0, 50, 1, psf_crop=64)
    import oracle
    ab, wb, _ = oracle.psf_fit(f.psf)
    o = a4.Oracle2004(f.dirty, f.psf, ab, wb, gain=0.3, smooth_scales=4, lm_max_iter=40)
    for _ in range(3):
        rep = o.step()
        assert rep["status"] in ("ok", "not_converged")
    want = rf.refreshed_residual(f.dirty, f.psf, o.components(), ab, wb)
    assert np.abs(o.R - want).max() <= 1e-10 * np.abs(f.dirty).max()


def test_stop_rules():
    wb = 1.5
    psf = psf_of([(1.0, wb, 0, 0)], 33)
    D = skygen.isolated_gaussian(32, 32, 0.5, 15.0, 16.0, 2.0)
    o = a4.Oracle2004(D, psf, 1.0, wb, threshold=0.6)
    assert o.step()["status"] == "threshold" and o.k == 0
    o = a4.Oracle2004(D, psf, 1.0, wb, max_iter=0)
    assert o.step()["status"] == "maxiter"
