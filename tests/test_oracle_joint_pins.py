"""Pins of the oracle's joint fit of an active set of two or more members
(Sect. 3, Eq. 4 over the members' windows, old members added back to the data).

Each test checks the oracle against something other than itself:
* the objective, its gradient and J^T J against a dense whole-image NumPy
  evaluation written here from the definitions, and against central finite
  differences of that dense model;
* exact recovery of overlapping noise-free Gaussians when the old members
  start from perturbed stored parameters (the add-back and the cross-member
  terms must all be right for the residual to vanish);
* the two-member LM optimum against a brute-force search with the amplitudes
  solved linearly.
A dropped add-back of the old members, dropped cross-member Gram blocks or a
union of windows that counts a pixel twice each fail at least one of these.
CPU only.
"""
import math

import numpy as np
import pytest
import scipy.optimize


def window(x, y, s, H, W, cw=5.0):
    """Half-width max(3, ceil(c_w s)) around the rounded centre, clipped."""
    h = max(3, math.ceil(cw * s))
    cx, cy = math.floor(x + 0.5), math.floor(y + 0.5)
    return max(0, cy - h), min(H - 1, cy + h), max(0, cx - h), min(W - 1, cx + h)


def dense_member(th, H, W):
    """G on the member's own window (zero elsewhere), its mask, and the four
    partial derivatives dG/d(a, x, y, s) from the closed form of a circular
    Gaussian a exp(-((c-x)^2 + (r-y)^2) / (2 s^2))."""
    a, x, y, s = th
    r0, r1, c0, c1 = window(x, y, s, H, W)
    mask = np.zeros((H, W), bool)
    mask[r0:r1 + 1, c0:c1 + 1] = True
    rr, cc = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = cc - x, rr - y
    q = dx * dx + dy * dy
    e = np.exp(-q / (2 * s * s))
    G = a * e
    J = np.stack([e, G * dx / s ** 2, G * dy / s ** 2, G * q / s ** 3]) * mask
    return G * mask, mask, J


def dense_eval(R, theta, stored):
    """F, H, g, chi2, |U| of the fit objective from the whole image."""
    H_, W_ = R.shape
    theta = np.asarray(theta, float)
    D = R.astype(np.float64).copy()
    for j in range(1, len(theta)):
        Gs, _, _ = dense_member(stored[j], H_, W_)
        D += Gs
    M = np.zeros_like(D)
    U = np.zeros(D.shape, bool)
    Js = []
    for th in theta:
        G, mask, J = dense_member(th, H_, W_)
        M += G
        U |= mask
        Js.append(J)
    J = np.concatenate(Js)[:, U]                   # n x |U|
    res = (D - M)[U]
    F = float((M * (M - 2 * D)).sum())             # M = 0 outside U
    return {"F": F, "H": J @ J.T, "g": J @ res, "chi2": float(res @ res), "npx": int(U.sum()),
            "M": M, "U": U}


def make_state(orc, R, wb=1.2, lm_tol=1e-5):
    return orc.Oracle(np.asarray(R, float), gain=1.0, max_iter=10, max_active=5,
                      alpha_b=1.0, omega_b=wb, lm_tol=lm_tol)


CASES = {
    # two members with overlapping windows
    "m2": ([[0.9, 20.3, 21.6, 2.1], [0.5, 24.8, 19.2, 1.63]],
           [[0, 0, 0, 0], [0.45, 25.1, 19.4, 1.7]]),
    # three members, one window clipped by the top edge, stored windows that
    # differ from the trial windows
    "m3": ([[0.9, 20.3, 21.6, 2.1], [0.5, 24.8, 19.2, 1.63], [-0.3, 18.2, 4.4, 1.3]],
           [[0, 0, 0, 0], [0.45, 25.1, 19.4, 1.7], [-0.35, 17.6, 3.9, 1.1]]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fit_eval_matches_dense_definition(orc, case):
    theta, stored = CASES[case]
    rng = np.random.default_rng(3)
    R = rng.normal(0, 0.2, size=(40, 36))
    o = make_state(orc, R)
    got = o.fit_eval(theta, stored)
    ref = dense_eval(R, theta, np.asarray(stored, float))
    assert got["npx"] == ref["npx"]
    assert got["F"] == pytest.approx(ref["F"], rel=1e-12, abs=1e-12)
    assert got["chi2"] == pytest.approx(ref["chi2"], rel=1e-12)
    scale = np.abs(ref["H"]).max()
    np.testing.assert_allclose(got["H"], ref["H"], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(got["g"], ref["g"], rtol=0, atol=1e-12 * np.abs(ref["g"]).max())
    # the cross-member blocks are not zero in these cases
    assert np.abs(ref["H"][0:4, 4:8]).max() > 1e-3 * scale


@pytest.mark.parametrize("case", sorted(CASES))
def test_fit_eval_finite_differences(orc, case):
    """g = -dF/dtheta / 2 and J^T J from central differences of the dense
    model, with steps small enough that no window moves."""
    theta, stored = CASES[case]
    theta = np.asarray(theta, float)
    rng = np.random.default_rng(4)
    R = rng.normal(0, 0.2, size=(40, 36))
    o = make_state(orc, R)
    got = o.fit_eval(theta, stored)
    n = theta.size
    h = 1e-6
    U = dense_eval(R, theta, np.asarray(stored, float))["U"]
    Jfd = np.zeros((n, int(U.sum())))
    for i in range(n):
        tp, tm = theta.copy().ravel(), theta.copy().ravel()
        tp[i] += h
        tm[i] -= h
        Fp = o.fit_eval(tp.reshape(-1, 4), stored)["F"]
        Fm = o.fit_eval(tm.reshape(-1, 4), stored)["F"]
        assert -(Fp - Fm) / (2 * h) / 2 == pytest.approx(got["g"][i], rel=1e-5, abs=1e-7)
        Mp = dense_eval(R, tp.reshape(-1, 4), np.asarray(stored, float))["M"]
        Mm = dense_eval(R, tm.reshape(-1, 4), np.asarray(stored, float))["M"]
        Jfd[i] = ((Mp - Mm) / (2 * h))[U]
    Hfd = Jfd @ Jfd.T
    np.testing.assert_allclose(got["H"], Hfd, rtol=0, atol=1e-6 * np.abs(Hfd).max())


def truncated(H, W, th):
    return dense_member(th, H, W)[0]


def test_joint_exact_recovery_from_perturbed_old_members(orc):
    """Three overlapping noise-free Gaussians; the component list holds two of
    them at perturbed parameters and the residual is the sky minus those.  With
    gain 1 one iteration fits the new component and refits both old members
    exactly, and the residual vanishes."""
    H = W = 64
    wb = 1.2
    A = [0.8, 30.3, 31.6, 3.0]
    B = [0.6, 35.6, 28.4, 2.2]
    C = [1.0, 31.2, 27.1, 1.6]
    A0 = [0.72, 30.6, 31.4, 3.15]
    B0 = [0.66, 35.9, 28.2, 2.3]
    sky = truncated(H, W, A) + truncated(H, W, B) + truncated(H, W, C)
    R = sky - truncated(H, W, A0) - truncated(H, W, B0)
    # a tight step tolerance, so that the fit ends at the optimum to rounding
    o = make_state(orc, R, wb=wb, lm_tol=1e-10)
    o.load_state(R, np.array([A0, B0]), 2)
    rep = o.step()
    assert rep["members"] == [-1, 1, 0]              # most recent first
    assert rep["converged"]
    np.testing.assert_allclose(rep["theta"], [C, B, A], rtol=1e-10, atol=1e-10)
    comps = o.comps()
    np.testing.assert_allclose(comps, [A, B, C], rtol=1e-10, atol=1e-10)
    assert np.abs(o.R).max() <= 1e-10


def test_two_member_lm_optimum_vs_brute_force(orc):
    """Two overlapping Gaussians plus noise on a 12 x 12 image, windows wider
    than the image: the LM optimum against Nelder-Mead over the six nonlinear
    parameters with both amplitudes solved by linear least squares."""
    rng = np.random.default_rng(21)
    H = W = 12
    rr, cc = np.mgrid[0:H, 0:W].astype(float)

    def g(x, y, s):
        return np.exp(-((cc - x) ** 2 + (rr - y) ** 2) / (2 * s * s))

    img = 1.0 * g(4.3, 5.2, 1.7) + 0.6 * g(7.4, 6.1, 2.0) + rng.normal(0, 0.01, (H, W))

    def chi2(p):
        x1, y1, s1, x2, y2, s2 = p
        B = np.stack([g(x1, y1, s1).ravel(), g(x2, y2, s2).ravel()], axis=1)
        amp, *_ = np.linalg.lstsq(B, img.ravel(), rcond=None)
        r = img.ravel() - B @ amp
        return float(r @ r), amp

    theta, trials, conv, c2 = orc.fit_gaussians(
        img, [[0.9, 4.0, 5.0, 1.5], [0.5, 7.0, 6.0, 1.5]], omega_b=1.0, max_width=10.0,
        window_sigmas=50.0)
    assert conv
    best = None
    for start in ([4.0, 5.0, 1.5, 7.0, 6.0, 1.5], [4.6, 5.5, 2.0, 7.8, 5.8, 1.7]):
        res = scipy.optimize.minimize(lambda p: chi2(p)[0], start, method="Nelder-Mead",
                                      options={"xatol": 1e-11, "fatol": 1e-15, "maxiter": 40000,
                                               "maxfev": 40000})
        if best is None or res.fun < best.fun:
            best = res
    x1, y1, s1, x2, y2, s2 = best.x
    a1, a2 = chi2(best.x)[1]
    assert c2 == pytest.approx(best.fun, rel=1e-8)
    np.testing.assert_allclose(theta, [[a1, x1, y1, s1], [a2, x2, y2, s2]], atol=2e-6)


def test_loop_gain_moves_old_members_toward_their_refit(orc):
    """Reading of the loop gain (Sect. 3) with an active set: every change of
    the model is scaled by the gain.  The fit itself does not depend on the
    gain (pinned above by exact recovery at gain 1); at gain g the new
    component joins with g times its amplitude and each old member moves the
    fraction g of the way to its refit; the residual is then the data minus
    the committed list, by definition."""
    H = W = 64
    A = [0.8, 30.3, 31.6, 3.0]
    B = [0.6, 35.6, 28.4, 2.2]
    C = [1.0, 31.2, 27.1, 1.6]
    A0 = np.array([0.72, 30.6, 31.4, 3.15])
    B0 = np.array([0.66, 35.9, 28.2, 2.3])
    sky = truncated(H, W, A) + truncated(H, W, B) + truncated(H, W, C)
    R = sky - truncated(H, W, A0) - truncated(H, W, B0)
    g = 0.35
    o = orc.Oracle(R, gain=g, max_iter=10, max_active=5, alpha_b=1.0, omega_b=1.2, lm_tol=1e-10)
    o.load_state(R, np.array([A0, B0]), 2)
    rep = o.step()
    assert rep["members"] == [-1, 1, 0] and rep["added"]
    np.testing.assert_allclose(rep["theta"], [C, B, A], rtol=1e-10, atol=1e-10)
    want = [A0 + g * (np.array(A) - A0), B0 + g * (np.array(B) - B0),
            [g * C[0], C[1], C[2], C[3]]]
    np.testing.assert_allclose(o.comps(), want, rtol=1e-12, atol=1e-12)
    expect = sky - sum(truncated(H, W, c) for c in want)
    assert np.abs(o.R - expect).max() <= 1e-12


def test_zero_amplitude_new_component_is_not_added(orc):
    """An old member that explains the peak: the residual is a Gaussian A
    minus a stored member at A's width, half its amplitude and 2 px off, less a
    small beam-sized dip at the peak, which lies 3 px from the stored centre
    (outside the co-location radius).  The joint fit moves the old member onto
    A, and the new component would need a negative amplitude: it stays on its
    sign bound 0.  It is not added: the list keeps one component, now the
    refit (gain 1), and the residual is the data minus that refit."""
    H = W = 64
    wb = 1.2
    A = [1.0, 30.0, 30.0, 4.0]
    A0 = [0.5, 32.0, 30.0, 4.0]
    dip = [0.005, 29.0, 30.0, wb]
    R = truncated(H, W, A) - truncated(H, W, A0) - truncated(H, W, dip)
    assert int(np.argmax(np.abs(R))) == 30 * W + 29
    o = orc.Oracle(R, gain=1.0, max_iter=10, max_active=5, alpha_b=1.0, omega_b=wb)
    o.load_state(R, np.array([A0]), 1)
    rep = o.step()
    assert rep["members"] == [-1, 0]
    assert rep["theta"][0][0] == 0.0 and not rep["added"]
    assert o.L == 1 and o.k == 2
    fit = rep["theta"][1]
    np.testing.assert_allclose(o.comps()[0], fit, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(fit, A, rtol=0, atol=0.02)
    expect = R + truncated(H, W, A0) - truncated(H, W, fit)
    assert np.abs(o.R - expect).max() <= 1e-12


def test_zero_amplitude_fit_from_a_proposal_falls_back(orc):
    """The state of the test above with a proposal near the peak (narrower
    than the old member) that beats the simple values at the start: LM from it
    converges to a new component of amplitude zero, a failed proposal, so the
    simple values are fitted instead.  The iteration then ends as the plain one
    does (same residual, same list), and its trial count holds both fits."""
    H = W = 64
    wb = 1.2
    A = [1.0, 30.0, 30.0, 4.0]
    A0 = [0.5, 32.0, 30.0, 4.0]
    dip = [0.005, 29.0, 30.0, wb]
    R = truncated(H, W, A) - truncated(H, W, A0) - truncated(H, W, dip)
    prop = [R[30, 29], 29.2, 30.0, 1.5]

    def fresh():
        o = orc.Oracle(R, gain=1.0, max_iter=10, max_active=5, alpha_b=1.0, omega_b=wb)
        o.load_state(R, np.array([A0]), 1)
        return o

    plain = fresh()
    rp = plain.step()
    o = fresh()
    rep = o.step(init=prop)
    assert rep["start_from_proposal"] and rep["used_fallback"] and rep["converged"]
    assert rep["theta"][0][0] == 0.0 and not rep["added"]
    assert rep["lm_iters"] > rp["lm_iters"]
    assert o.L == plain.L == 1
    np.testing.assert_array_equal(o.R, plain.R)
    np.testing.assert_array_equal(o.comps(), plain.comps())


def test_field_run_adds_no_zero_amplitude_component(orc):
    """On the 1024^2 EVLA-like field (seed 1000) the joint fits often leave the
    new component at zero amplitude, an old member explaining the peak; none
    of those is added, so no component of the list has amplitude zero and the
    list is shorter than the iteration count by exactly those iterations."""
    import skygen
    f = skygen.make_c1024(1000)
    ab, wb, _ = orc.psf_fit(f.psf)
    o = orc.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                   max_active=f.max_active, alpha_b=ab, omega_b=wb)
    skipped = 0
    for _ in range(150):
        rep = o.step()
        skipped += 0 if rep["added"] else 1
        assert rep["added"] == (rep["theta"][0][0] != 0.0)
    assert skipped >= 5
    assert o.L == 150 - skipped
    assert np.all(o.comps()[:, 0] != 0.0)
    assert np.abs(o.residual_from_scratch() - o.R).max() <= 1e-12 * np.abs(f.dirty).max()
