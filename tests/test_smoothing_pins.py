"""Pins of the smoothing-method oracle (oracle/smoothing.py): the initial
values of Sect. 2 step 1 and Sect. 3, and the switch between the smoothing and
the simple method (Sect. 3).  The checks come from outside the oracle: brute
force loops and least squares on tiny images, closed forms for isolated
Gaussians, invariances, and the switch's stated effect on the iteration."""
import math

import numpy as np
import pytest

import oracle
import skygen
from oracle import smoothing as sm

OMEGA_B = 1.3


def brute_corr(R, sigma, ws=5.0):
    """C and N by explicit loops over output pixel and window pixel."""
    H, W = R.shape
    h = max(3, math.ceil(ws * sigma))
    C = np.zeros((H, W))
    N = np.zeros((H, W))
    for r in range(H):
        for c in range(W):
            acc = nrm = 0.0
            for rr in range(max(0, r - h), min(H, r + h + 1)):
                for cc in range(max(0, c - h), min(W, c + h + 1)):
                    k = math.exp(-((rr - r) ** 2 + (cc - c) ** 2) / (2.0 * sigma * sigma))
                    acc += k * R[rr, cc]
                    nrm += k * k
            C[r, c], N[r, c] = acc, nrm
    return C, N


@pytest.mark.parametrize("shape,sigma", [((7, 11), 0.8), ((9, 6), 1.3), ((5, 13), 2.6)])
def test_both_evaluations_match_the_window_sums(shape, sigma):
    """Small ragged images whose windows reach past every edge."""
    R = np.random.default_rng(3).normal(size=shape)
    C0, N0 = brute_corr(R, sigma)
    for method in ("direct", "fft"):
        C, N = sm.smoothed(R, sigma, method=method)
        assert np.abs(C - C0).max() <= 1e-12 * np.abs(C0).max(), method
        assert np.abs(N - N0).max() <= 1e-12 * N0.max(), method


def test_l2_score_is_the_least_squares_drop():
    """With the l2 reading, S^2 is the drop of the squared residual when the
    least-squares multiple of the window's Gaussian is removed, and C/N is
    that multiple (numpy lstsq on every window of a tiny image)."""
    R = np.random.default_rng(5).normal(size=(8, 9))
    H, W = R.shape
    for sigma, C, N, S in sm.scores(R, 0.7, 3, 10.0, method="direct", norm="l2"):
        h = sm.halfwidth(sigma)
        for r in range(H):
            for c in range(W):
                r0, r1, c0, c1 = max(0, r - h), min(H, r + h + 1), max(0, c - h), min(W, c + h + 1)
                yy, xx = np.mgrid[r0:r1, c0:c1]
                g = np.exp(-((yy - r) ** 2 + (xx - c) ** 2) / (2 * sigma * sigma)).ravel()
                d = R[r0:r1, c0:c1].ravel()
                a, *_ = np.linalg.lstsq(g[:, None], d, rcond=None)
                drop = d @ d - np.sum((d - a[0] * g) ** 2)
                assert abs(a[0] - C[r, c] / N[r, c]) <= 1e-10 * max(1.0, abs(a[0]))
                assert abs(drop - S[r, c] ** 2) <= 1e-10 * max(1.0, drop)


@pytest.mark.parametrize("j", [0, 1, 2, 3])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_l2_recovers_an_isolated_gaussian_of_a_trial_width(j, sign):
    """A Gaussian of exactly a trial width, centred on a pixel: the l2 peak is
    that width at that pixel and the amplitude is exact (the residual on the
    window is that multiple of the kernel)."""
    sig = OMEGA_B * 2 ** j
    n = 2 * sm.halfwidth(sig) + 41
    x0, y0 = n // 2 + 3, n // 2 - 5
    R = skygen.isolated_gaussian(n, n, sign * 0.7, x0, y0, sig)
    b = sm.best(R, OMEGA_B, 4, 100.0, norm="l2")
    assert b["scale"] == j and b["idx"] == y0 * n + x0
    assert abs(b["start"][0] - sign * 0.7) <= 1e-12
    assert tuple(b["start"][1:]) == (x0, y0, sig)


def test_l2_recovers_a_gaussian_in_the_corner():
    """The clipped window's norm keeps the amplitude exact at the image corner."""
    sig = OMEGA_B * 2
    R = skygen.isolated_gaussian(40, 50, 1.5, 0.0, 0.0, sig)
    b = sm.best(R, OMEGA_B, 4, 100.0, norm="l2")
    assert b["scale"] == 1 and b["idx"] == 0
    assert abs(b["start"][0] - 1.5) <= 1e-12


@pytest.mark.parametrize("ratio,want", [(1.2, 0), (1.6, 1), (2.6, 1), (3.0, 2)])
def test_l2_scale_choice_follows_the_matched_filter(ratio, want):
    """A centred Gaussian of width s between two trial widths: the normalised
    response 2 s sigma / (s^2 + sigma^2) (continuous limit) is larger for
    sigma_j exactly when s < sqrt(sigma_j sigma_{j+1})."""
    s = OMEGA_B * ratio
    n = 101
    R = skygen.isolated_gaussian(n, n, 1.0, 50.0, 50.0, s)
    b = sm.best(R, OMEGA_B, 4, 100.0, norm="l2")
    assert b["scale"] == want and b["idx"] == 50 * n + 50


def test_peak_norm_prefers_the_widest_beam_and_its_amplitude():
    """With peak-1 beams, smoothing a centred Gaussian of width s with width
    sigma gives 2 pi a s^2 sigma^2 / (s^2 + sigma^2) at the centre, growing
    with sigma: the widest beam wins, and the least-squares amplitude there is
    2 a s^2 / (s^2 + sigma^2)."""
    s, a = 2.0, 0.8
    n = 2 * sm.halfwidth(OMEGA_B * 8) + 21
    c = n // 2
    R = skygen.isolated_gaussian(n, n, a, c, c, s)
    b = sm.best(R, OMEGA_B, 4, 100.0, norm="peak")
    sig = OMEGA_B * 8
    assert b["scale"] == 3 and b["idx"] == c * n + c
    want_c = 2 * math.pi * a * s * s * sig * sig / (s * s + sig * sig)
    assert abs(b["corr"] - want_c) <= 1e-6 * want_c
    want_a = 2 * a * s * s / (s * s + sig * sig)
    assert abs(b["start"][0] - want_a) <= 1e-6 * want_a


@pytest.mark.parametrize("norm", sm.NORMS)
def test_invariances(norm):
    rng = np.random.default_rng(9)
    R = rng.normal(size=(40, 37))
    b = sm.best(R, OMEGA_B, 3, 100.0, norm=norm)
    b2 = sm.best(-2.5 * R, OMEGA_B, 3, 100.0, norm=norm)
    assert (b2["scale"], b2["idx"]) == (b["scale"], b["idx"])
    assert abs(b2["start"][0] + 2.5 * b["start"][0]) <= 1e-12 * abs(b["start"][0]) * 2.5
    # a feature far from the edges moves with a shift of the image
    Z = np.zeros((90, 90))
    G = skygen.isolated_gaussian(31, 31, 1.0, 15.0, 15.0, 2.0)
    Z[10:41, 20:51] = G
    Z2 = np.zeros((90, 90))
    Z2[30:61, 25:56] = G
    p = sm.best(Z, OMEGA_B, 2, 100.0, norm=norm)
    q = sm.best(Z2, OMEGA_B, 2, 100.0, norm=norm)
    assert p["scale"] == q["scale"] and q["idx"] - p["idx"] == 20 * 90 + 5
    assert abs(p["start"][0] - q["start"][0]) <= 1e-12


def test_ties_and_the_zero_image():
    Z = np.zeros((20, 30))
    b = sm.best(Z, OMEGA_B, 3, 100.0)
    assert b["scale"] == 0 and b["idx"] == 0 and b["start"][0] == 0.0
    # two equal features: the lower row-major index wins
    R = np.zeros((60, 60))
    g = skygen.isolated_gaussian(21, 21, 1.0, 10.0, 10.0, 1.5)
    R[5:26, 30:51] = g
    R[30:51, 5:26] = g
    b = sm.best(R, OMEGA_B, 2, 100.0, method="direct")
    assert b["idx"] == 15 * 60 + 40


def test_widths():
    assert sm.widths(1.5, 5, 100.0) == [1.5, 3.0, 6.0, 12.0, 24.0]
    assert sm.widths(1.5, 5, 7.0) == [1.5, 3.0, 6.0]
    assert sm.widths(1.5, 5, 1.0) == [1.5]


def test_switch_rule_areas():
    # convolved areas: 5 % of pi s0^2 is reached at s = sqrt(0.05) s0 = 0.2236 s0
    assert sm.simple_next(0.22 * 10.0, 10.0, 1.3)
    assert not sm.simple_next(0.23 * 10.0, 10.0, 1.3)
    # a simple start has s0 = omega_b and the fit keeps s >= omega_b
    assert not sm.simple_next(1.3, 1.3, 1.3)
    # deconvolved areas: a point-like fit from a wider start
    assert sm.simple_next(1.3, 2.6, 1.3, deconvolved=True)
    assert not sm.simple_next(1.3, 1.3, 1.3, deconvolved=True)


def test_start_values_drive_the_fit():
    """A step from a start at the exact parameters of an isolated Gaussian
    keeps them: the fit's first point is already the minimum."""
    n, sig = 64, 3.0
    R = skygen.isolated_gaussian(n, n, 0.9, 30.0, 33.0, sig)
    o = oracle.Oracle(R, gain=1.0, threshold=0.0, max_iter=5, max_active=3, alpha_b=1.0,
                      omega_b=OMEGA_B, smooth_scales=3)
    rep = o.step(start=[0.9, 30.0, 33.0, sig])
    assert rep["smoothed"] and rep["converged"]
    assert np.abs(rep["theta0"][0] - [0.9, 30.0, 33.0, sig]).max() == 0.0
    assert np.abs(rep["theta"][0] - [0.9, 30.0, 33.0, sig]).max() <= 1e-9
    assert np.abs(o.R).max() <= 1e-6


def test_switch_sequence_on_a_field():
    """On a 128 x 128 field with peak-1 beams: the first iteration smooths, an
    iteration uses the simple method exactly when the previous fit shrank the
    new component below 5 % of its start area, a simple iteration is followed
    by a smoothing one, and a smoothing iteration starts from the oracle's own
    smoothing peak."""
    f = skygen.make_c128(0)
    ab, wb, _ = oracle.psf_fit(f.psf)
    o = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active, alpha_b=ab, omega_b=wb, smooth_scales=4)
    prev = None
    n_simple = 0
    for it in range(70):
        R0 = o.R.copy()
        rep = o.step()
        assert rep["status"] in (0, 3)
        if prev is None:
            assert rep["smoothed"]
        else:
            due = sm.simple_next(prev["theta"][0, 3], prev["theta0"][0, 3], wb)
            assert rep["smoothed"] == (not due), it
            if not prev["smoothed"]:
                assert rep["smoothed"]
        if rep["smoothed"]:
            b = sm.best(R0, wb, 4, o.s_max)
            assert np.abs(rep["theta0"][0] - b["start"]).max() <= 1e-12 * max(1.0, abs(b["start"][0]))
        else:
            n_simple += 1
            r, c = divmod(rep["idx"], f.shape[1])
            assert tuple(rep["theta0"][0]) == (R0.flat[rep["idx"]], c, r, wb)
        prev = rep
    assert n_simple >= 1
