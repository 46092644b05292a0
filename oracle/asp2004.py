"""FP64 oracle of the Asp-Clean2004 iteration -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP library.

What it computes (Sect. 2, steps 1-4 with the objective of Eq. 3): the
comparison path against which the paper measures Asp-Clean2016 (Table 3).  An
iteration

1. takes the start values from the smoothing method (Sect. 2 step 1; the
   2004 algorithm smooths in every iteration, there is no switch);
2. fits the new component in the sky plane by Levenberg-Marquardt, with the
   objective chi^2 = || R - B (*) g(theta) ||^2 over the whole image (Eq. 3
   with the earlier components fixed, so that the data is the current
   residual R), where B is the true PSF and the convolution is carried out in
   every evaluation (here SciPy's FFT, a library primitive);
3. adds the component with the loop gain and subtracts its PSF-convolved
   image from the residual (Sect. 2 step 3, exact: R stays
   I_dirty - B (*) I_model);
4. stops on the threshold or the iteration count (Sect. 2 step 4).

Readings where the paper is silent (each listed in the design notes):

* The parameters are theta = (F, x, y, v): flux, centre and the squared width
  v = omega^2 of the sky component.  The component image g(theta) is rendered
  as the exact-PSF refresh renders the model (``oracle/refresh.py``): a
  sampled Gaussian for omega >= 1 px, Gauss-Hermite nodes spread by Lanczos-3
  below.  That rendering is even in omega, so its derivative in omega vanishes
  at a point source and a fit there cannot leave the bound omega = 0; in v the
  derivative is finite and in general not zero (at v = 0 it is half the
  second derivative of the profile).  The Jacobian columns are
  B (*) dg/dtheta_k with the derivatives of the rendering taken analytically
  in the regime of the current width.
* One component is fitted per iteration (the paper's cost count is for a
  single component); the earlier ones stay fixed.
* Start: from the smoothing start (a_c, col, row, sigma_j) in convolved space,
  v_0 = max(sigma_j^2 - omega_b^2, 0) and, by Eq. 5,
  F_0 = a_c sigma_j^2 / (alpha_b omega_b^2).
* Bounds: F keeps the start's sign; x and y stay in the window of the start
  (half-width max(3, ceil(c_w s_0)), s_0 = sqrt(v_0 + omega_b^2)); v in
  [0, max(s_max^2 - omega_b^2, 0)], s_max the width bound of the
  Asp-Clean2016 fit.
* LM: the rules of the Asp-Clean2016 fit (the C oracle's ``lm_fit``) restated
  for four parameters, with F(theta) = sum over the image of m (m - 2 R),
  m = B (*) g(theta), which is chi^2 less the constant sum of R^2; the step
  test scales x and y by s = sqrt(v + omega_b^2) and v by s^2.
* The component is kept in the list in convolved-space form, the Gaussian
  (a, s) whose Eqs. 5-6 deconvolution is (gain F, omega), so the reported
  components and the exact-PSF refresh read it like any other.
"""
from __future__ import annotations

import math

import numpy as np

from . import refresh as rf
from . import smoothing as sm

MU_MIN, MU_MAX = 1e-12, 1e8
SMALL_WIDTH = 1e-4               # px: below, dg/dv takes its limit at omega = 0


# ---------------------------------------------------------------------------
# The component image and its derivatives
# ---------------------------------------------------------------------------

def _dsinc(t: np.ndarray) -> np.ndarray:
    """d/dt of sin(pi t) / (pi t)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = np.abs(t) < 1e-3
    ts = t[small]
    pi2 = math.pi * math.pi
    out[small] = -pi2 * ts / 3.0 + pi2 * pi2 * ts ** 3 / 30.0
    tb = t[~small]
    out[~small] = (np.cos(math.pi * tb) - np.sinc(tb)) / tb
    return out


def _d2sinc(t: np.ndarray) -> np.ndarray:
    """d^2/dt^2 of sin(pi t) / (pi t)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = np.abs(t) < 1e-3
    ts = t[small]
    pi2 = math.pi * math.pi
    out[small] = -pi2 / 3.0 + pi2 * pi2 * ts * ts / 10.0
    tb = t[~small]
    out[~small] = -pi2 * np.sinc(tb) - 2.0 * _dsinc(tb) / tb
    return out


def lanczos_deriv(t: np.ndarray) -> np.ndarray:
    """d/dt of the Lanczos-3 kernel sinc(t) sinc(t/3), zero for |t| >= 3."""
    t = np.asarray(t, dtype=np.float64)
    d = _dsinc(t) * np.sinc(t / 3.0) + np.sinc(t) * _dsinc(t / 3.0) / 3.0
    return np.where(np.abs(t) < rf.LANCZOS_A, d, 0.0)


def lanczos_deriv2(t: np.ndarray) -> np.ndarray:
    """d^2/dt^2 of the Lanczos-3 kernel, zero for |t| >= 3."""
    t = np.asarray(t, dtype=np.float64)
    u = t / 3.0
    d = (_d2sinc(t) * np.sinc(u) + 2.0 * _dsinc(t) * _dsinc(u) / 3.0 +
         np.sinc(t) * _d2sinc(u) / 9.0)
    return np.where(np.abs(t) < rf.LANCZOS_A, d, 0.0)


def _axis(x: float, v: float):
    """First pixel, normalised weights w and dw/dx, dw/dv (v = omega^2) of one
    axis of the interpolated profile (the refresh's narrow-component
    rendering)."""
    omega = math.sqrt(v)
    c0 = int(math.floor(x)) - 5
    cs = np.arange(c0, c0 + 12, dtype=np.float64)
    u = np.zeros_like(cs)
    ux = np.zeros_like(cs)
    uv = np.zeros_like(cs)
    for d, p in zip(rf.GH_OFFSETS, rf.GH_WEIGHTS):
        t = cs - x - d * omega
        u += p * rf.lanczos(t)
        ld = lanczos_deriv(t)
        ux -= p * ld
        if omega >= SMALL_WIDTH:
            uv -= p * d * ld / (2.0 * omega)
    if omega < SMALL_WIDTH:
        # the limit: sum_k p_k d_k^2 L''(t) / 2, and sum_k p_k d_k^2 = 1
        uv = 0.5 * lanczos_deriv2(cs - x)
    S = u.sum()
    w = u / S
    wx = (ux - w * ux.sum()) / S
    wv = (uv - w * uv.sum()) / S
    return c0, w, wx, wv


def unit_images(shape, x: float, y: float, v: float, window_sigmas: float = 5.0):
    """(g, dg/dx, dg/dy, dg/dv) of the unit-flux component at (x, y) of squared
    width v on the H x W grid, zero outside its footprint."""
    H, W = shape
    g = np.zeros((H, W))
    gx = np.zeros((H, W))
    gy = np.zeros((H, W))
    gv = np.zeros((H, W))
    omega = math.sqrt(v)
    if omega >= rf.RENDER_MIN_WIDTH:
        h = rf.halfwidth(omega, window_sigmas)
        cx, cy = int(math.floor(x + 0.5)), int(math.floor(y + 0.5))
        r0, r1 = max(0, cy - h), min(H - 1, cy + h)
        c0, c1 = max(0, cx - h), min(W - 1, cx + h)
        if r0 > r1 or c0 > c1:
            return g, gx, gy, gv
        dy = np.arange(r0, r1 + 1, dtype=np.float64)[:, None] - y
        dx = np.arange(c0, c1 + 1, dtype=np.float64)[None, :] - x
        q = dx * dx + dy * dy
        e = np.exp(-q / (2.0 * v)) / (2.0 * math.pi * v)
        sl = (slice(r0, r1 + 1), slice(c0, c1 + 1))
        g[sl] = e
        gx[sl] = e * dx / v
        gy[sl] = e * dy / v
        gv[sl] = e * (q / (2.0 * v * v) - 1.0 / v)
        return g, gx, gy, gv
    cx0, wx, dwx, wvx = _axis(x, v)
    cy0, wy, dwy, wvy = _axis(y, v)
    for i in range(12):
        r = cy0 + i
        if r < 0 or r >= H:
            continue
        for j in range(12):
            c = cx0 + j
            if c < 0 or c >= W:
                continue
            g[r, c] = wy[i] * wx[j]
            gx[r, c] = wy[i] * dwx[j]
            gy[r, c] = dwy[i] * wx[j]
            gv[r, c] = wvy[i] * wx[j] + wy[i] * wvx[j]
    return g, gx, gy, gv


# ---------------------------------------------------------------------------
# Eq. 3 and its Levenberg-Marquardt fit
# ---------------------------------------------------------------------------

class Problem:
    """chi^2(theta) = || R - B (*) g(theta) ||^2 on the whole image."""

    def __init__(self, R, psf, omega_b: float, window_sigmas: float = 5.0):
        self.R = np.asarray(R, dtype=np.float64)
        self.psf = np.asarray(psf, dtype=np.float64)
        self.omega_b = float(omega_b)
        self.ws = float(window_sigmas)
        self.evaluations = 0

    def convolved(self, theta):
        """B (*) g(theta) (with its flux)."""
        F, x, y, v = (float(t) for t in theta)
        g = unit_images(self.R.shape, x, y, v, self.ws)[0]
        return F * rf.convolve_psf(g, self.psf)

    def evaluate(self, theta, want_jac: bool = True):
        """(F(theta), chi^2, J^T J, J^T r) with F = sum m (m - 2 R), r = R - m."""
        self.evaluations += 1
        F, x, y, v = (float(t) for t in theta)
        imgs = unit_images(self.R.shape, x, y, v, self.ws)
        conv = [rf.convolve_psf(im, self.psf) for im in (imgs if want_jac else imgs[:1])]
        m = F * conv[0]
        r = self.R - m
        obj = float(np.sum(m * (m - 2.0 * self.R)))
        chi2 = float(np.sum(r * r))
        if not want_jac:
            return obj, chi2, None, None
        J = np.stack([conv[0].ravel(), F * conv[1].ravel(), F * conv[2].ravel(),
                      F * conv[3].ravel()], axis=1)
        return obj, chi2, J.T @ J, J.T @ r.ravel()


def _cholesky_solve(A: np.ndarray, b: np.ndarray):
    """Solve A x = b for symmetric positive definite A; None if A is not."""
    n = A.shape[0]
    Lm = np.zeros_like(A)
    for i in range(n):
        for k in range(i + 1):
            s = A[i, k] - float(np.dot(Lm[i, :k], Lm[k, :k]))
            if i == k:
                if not (s > 0.0):
                    return None
                Lm[i, i] = math.sqrt(s)
            else:
                Lm[i, k] = s / Lm[k, k]
    z = np.zeros(n)
    for i in range(n):
        z[i] = (b[i] - float(np.dot(Lm[i, :i], z[:i]))) / Lm[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (z[i] - float(np.dot(Lm[i + 1:, i], x[i + 1:]))) / Lm[i, i]
    return x


def lm_fit(prob: Problem, theta0, lo, hi, budget: int = 100, mu0: float = 1e-3,
           tol: float = 1e-5) -> dict:
    """Levenberg-Marquardt with the Asp-Clean2016 fit's rules: damped system
    (H + mu D) delta = g, D = diag(max(H_ii, 1e-12 max H_ii)); a parameter on a
    bound with its gradient pointing out is held for the trial; the trial is
    clipped to the bounds and accepted iff F decreases; gain-ratio damping
    (Madsen, Nielsen & Tingleff); converged on an accepted step with
    max |delta_k| / scale_k < tol (scales |F|, s, s, s^2 with
    s = sqrt(v + omega_b^2)), or stalled once mu passes 1e8; the budget counts
    trials."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    theta = np.clip(np.asarray(theta0, dtype=np.float64), lo, hi)
    Fv, chi2, Hs, g = prob.evaluate(theta)
    out = {"theta0": theta.copy(), "chi2_init": chi2, "F0": Fv}
    mu, nu = mu0, 2.0
    trials, converged = 0, False
    while trials < budget:
        dmax = float(np.max(np.diag(Hs)))
        dd = np.maximum(np.diag(Hs), 1e-12 * dmax)
        A = Hs + np.diag(mu * dd)
        rhs = g.copy()
        for i in range(4):
            if (theta[i] <= lo[i] and g[i] <= 0.0) or (theta[i] >= hi[i] and g[i] >= 0.0):
                A[i, :] = 0.0
                A[:, i] = 0.0
                A[i, i] = 1.0
                rhs[i] = 0.0
        trials += 1
        delta = _cholesky_solve(A, rhs)
        Ft = math.inf
        if delta is not None:
            pred = float(np.sum(delta * (rhs + mu * dd * delta)))
            trial = np.clip(theta + delta, lo, hi)
            Ft, chi2t, Ht, gt = prob.evaluate(trial)
            if not math.isfinite(Ft):
                Ft = math.inf
        if Ft < Fv:
            s2 = trial[3] + prob.omega_b * prob.omega_b
            st = math.sqrt(s2)
            sa = max(abs(trial[0]), 1e-30)
            step = max(abs(trial[0] - theta[0]) / sa, abs(trial[1] - theta[1]) / st,
                       abs(trial[2] - theta[2]) / st, abs(trial[3] - theta[3]) / s2)
            rho = (Fv - Ft) / pred if pred > 0.0 else 1.0
            t = 2.0 * rho - 1.0
            mu *= max(1.0 / 3.0, 1.0 - t * t * t)
            mu = max(mu, MU_MIN)
            nu = 2.0
            theta, Fv, chi2, Hs, g = trial, Ft, chi2t, Ht, gt
            if step < tol:
                converged = True
                break
        else:
            mu *= nu
            nu *= 2.0
            if mu > MU_MAX:
                converged = True
                break
    out.update({"theta": theta, "F": Fv, "chi2_final": chi2, "trials": trials,
                "converged": converged, "hess": Hs, "grad": g})
    return out


# ---------------------------------------------------------------------------
# The iteration
# ---------------------------------------------------------------------------

def start_from_smoothing(start4, alpha_b: float, omega_b: float):
    """Sky-plane (F, x, y, v = omega^2) from the smoothing start (a_c, col, row,
    sigma)."""
    a_c, x, y, s = (float(v) for v in start4)
    v = max(s * s - omega_b * omega_b, 0.0)
    return np.array([a_c * s * s / (alpha_b * omega_b * omega_b), x, y, v])


def convolved_form(F: float, omega: float, alpha_b: float, omega_b: float):
    """The Gaussian (a, s) whose Eqs. 5-6 deconvolution is (F, omega)."""
    s = math.sqrt(omega * omega + omega_b * omega_b)
    return F * alpha_b * omega_b * omega_b / (s * s), s


class Oracle2004:
    """The FP64 Asp-Clean2004 iteration on a residual it owns."""

    def __init__(self, dirty, psf, alpha_b: float, omega_b: float, *, gain=0.1, threshold=0.0,
                 max_iter=1000, lm_max_iter=100, window_sigmas=5.0, lm_tol=1e-5, lm_mu0=1e-3,
                 max_width=0.0, smooth_scales=5, smooth_norm="peak"):
        self.dirty = np.asarray(dirty, dtype=np.float64)
        self.psf = np.asarray(psf, dtype=np.float64)
        self.R = self.dirty.copy()
        self.alpha_b, self.omega_b = float(alpha_b), float(omega_b)
        self.gain, self.threshold = float(gain), float(threshold)
        self.max_iter, self.lm_max_iter = int(max_iter), int(lm_max_iter)
        self.ws, self.tol, self.mu0 = float(window_sigmas), float(lm_tol), float(lm_mu0)
        H, W = self.dirty.shape
        m = max_width if max_width > 0.0 else min(H, W) / 8.0
        self.s_max = max(m, self.omega_b)
        self.smooth_scales, self.smooth_norm = int(smooth_scales), smooth_norm
        self.comps: list[list[float]] = []
        self.k = 0

    def load_state(self, R, comps, k):
        self.R = np.asarray(R, dtype=np.float64).reshape(self.dirty.shape).copy()
        self.comps = [list(map(float, c)) for c in np.asarray(comps, dtype=np.float64).reshape(-1, 4)]
        self.k = int(k)

    def bounds(self, theta0):
        H, W = self.R.shape
        s0 = math.sqrt(theta0[3] + self.omega_b ** 2)
        h = rf.halfwidth(s0, self.ws)
        cx, cy = int(math.floor(theta0[1] + 0.5)), int(math.floor(theta0[2] + 0.5))
        r0, r1 = max(0, cy - h), min(H - 1, cy + h)
        c0, c1 = max(0, cx - h), min(W - 1, cx + h)
        neg = theta0[0] < 0.0
        v_max = max(self.s_max ** 2 - self.omega_b ** 2, 0.0)
        lo = [-math.inf if neg else 0.0, float(c0), float(r0), 0.0]
        hi = [0.0 if neg else math.inf, float(c1), float(r1), v_max]
        return lo, hi

    def step(self, start=None, method=None) -> dict:
        """One iteration; ``start`` overrides the smoothing start (a_c, col, row,
        sigma) when the caller checked a near tie."""
        R = self.R
        flat = np.abs(R).ravel()
        idx = int(np.argmax(flat))          # the first maximum: lowest index on ties
        pv = float(R.ravel()[idx])
        out = {"idx": idx, "peak": pv}
        if abs(pv) < self.threshold:
            out["status"] = "threshold"
            return out
        if self.k >= self.max_iter:
            out["status"] = "maxiter"
            return out
        sb = None
        if start is None:
            sb = sm.best(R, self.omega_b, self.smooth_scales, self.s_max, self.ws, method,
                         self.smooth_norm)
            start = sb["start"]
            out["smooth"] = {k: sb[k] for k in ("scale", "idx", "sigma", "score")}
        out["start_c"] = np.asarray(start, dtype=np.float64)
        th0 = start_from_smoothing(start, self.alpha_b, self.omega_b)
        lo, hi = self.bounds(th0)
        prob = Problem(R, self.psf, self.omega_b, self.ws)
        fit = lm_fit(prob, th0, lo, hi, self.lm_max_iter, self.mu0, self.tol)
        th = fit["theta"]
        conv = prob.convolved([self.gain * th[0], th[1], th[2], th[3]])
        self.R = R - conv
        a, s = convolved_form(self.gain * th[0], math.sqrt(th[3]), self.alpha_b, self.omega_b)
        self.comps.append([a, float(th[1]), float(th[2]), s])
        self.k += 1
        out.update({"status": "ok" if fit["converged"] else "not_converged",
                    "theta0": fit["theta0"], "theta": th, "trials": fit["trials"],
                    "converged": fit["converged"], "chi2_init": fit["chi2_init"],
                    "chi2_final": fit["chi2_final"], "evaluations": prob.evaluations,
                    "lo": lo, "hi": hi})
        return out

    def components(self) -> np.ndarray:
        return np.asarray(self.comps, dtype=np.float64).reshape(-1, 4)
