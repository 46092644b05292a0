"""FP64 oracle of the exact-PSF residual refresh -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP library.

What it computes (Sect. 2, step 3 of the Asp-Clean loop): the residual is the
dirty image minus the true PSF convolved with the model image,
R = I_dirty - B (*) I_model.  The minor cycle subtracts each component's
Gaussian main-lobe approximation (Sect. 3) on a window; a refresh replaces
that residual by the one of the definition, so that the sidelobes of every
component found so far leave the residual at once.

The model image (Sect. 2 step 2 writes it as a sum of sampled Gaussians) on
the pixel grid -- readings where the paper is silent:

* Each component enters with its deconvolved parameters (Eqs. 5-6): flux F,
  width omega, centre (x, y); the amplitude after the loop gain.
* omega >= 1 px: the Gaussian alpha exp(-|p - c|^2 / (2 omega^2)) sampled at
  pixel centres on the window of half-width max(3, ceil(c_w omega)) around
  the rounded centre, clipped to the image.
* omega < 1 px (points included): a Gaussian narrower than a pixel cannot be
  sampled; its flux is spread by band-limited interpolation.  Per axis, the
  3-point Gauss-Hermite rule of the Gaussian (offsets 0, +-sqrt(3) omega,
  weights 2/3, 1/6, 1/6) places three sub-pixel points, each spread with the
  Lanczos-3 kernel sinc(t) sinc(t/3) (|t| < 3); the per-axis weights are
  normalised to sum 1 and the component adds F w_y(r) w_x(c), clipped to the
  image.  For a band-limited PSF (an interferometric PSF is) this moves the
  PSF by the sub-pixel offset to the accuracy of the interpolation.
* The convolution is linear (zero outside the image), with the PSF centred
  on its peak pixel (the largest value, lowest index on ties): the dirty
  image's own convention.  Evaluated by SciPy's FFT (a library primitive).
"""
from __future__ import annotations

import math

import numpy as np

RENDER_MIN_WIDTH = 1.0           # px: narrower components are interpolated
GH_OFFSETS = (0.0, math.sqrt(3.0), -math.sqrt(3.0))   # in units of omega
GH_WEIGHTS = (2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0)
LANCZOS_A = 3


def deconvolve(a, s, alpha_b, omega_b):
    """Eqs. (5)-(6): (flux, alpha, omega, is_point) of a fitted Gaussian (a, s)."""
    flux = a * s * s / (alpha_b * omega_b * omega_b)
    w2 = s * s - omega_b * omega_b
    omega = math.sqrt(w2) if w2 > 0.0 else 0.0
    if omega > 1e-6 * omega_b:
        return flux, flux / (2.0 * math.pi * omega * omega), omega, False
    return flux, 0.0, 0.0, True


def lanczos(t: np.ndarray) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    out = np.where(np.abs(t) < LANCZOS_A, np.sinc(t) * np.sinc(t / LANCZOS_A), 0.0)
    return out


def axis_weights(x: float, omega: float):
    """(first pixel, weights) of the interpolated 1-D profile around x."""
    c0 = int(math.floor(x)) - 5
    cs = np.arange(c0, c0 + 12, dtype=np.float64)
    w = np.zeros_like(cs)
    for d, p in zip(GH_OFFSETS, GH_WEIGHTS):
        w += p * lanczos(cs - x - d * omega)
    return c0, w / w.sum()


def halfwidth(s: float, window_sigmas: float = 5.0) -> int:
    return int(max(3, math.ceil(window_sigmas * s)))


def model_image(shape, comps: np.ndarray, alpha_b: float, omega_b: float,
                window_sigmas: float = 5.0) -> np.ndarray:
    """The model image of the convolved-space component list (L, 4) = (a, x, y, s)."""
    H, W = shape
    M = np.zeros((H, W), dtype=np.float64)
    for a, x, y, s in np.asarray(comps, dtype=np.float64).reshape(-1, 4):
        F, alpha, omega, is_point = deconvolve(a, s, alpha_b, omega_b)
        if not is_point and omega >= RENDER_MIN_WIDTH:
            h = halfwidth(omega, window_sigmas)
            cx, cy = int(math.floor(x + 0.5)), int(math.floor(y + 0.5))
            r0, r1 = max(0, cy - h), min(H - 1, cy + h)
            c0, c1 = max(0, cx - h), min(W - 1, cx + h)
            if r0 > r1 or c0 > c1:
                continue
            rr = np.arange(r0, r1 + 1, dtype=np.float64)[:, None] - y
            cc = np.arange(c0, c1 + 1, dtype=np.float64)[None, :] - x
            M[r0:r1 + 1, c0:c1 + 1] += alpha * np.exp(-(rr * rr + cc * cc) / (2.0 * omega * omega))
        else:
            om = 0.0 if is_point else omega
            cx0, wx = axis_weights(x, om)
            cy0, wy = axis_weights(y, om)
            for i, wyv in enumerate(wy):
                r = cy0 + i
                if r < 0 or r >= H:
                    continue
                for j, wxv in enumerate(wx):
                    c = cx0 + j
                    if 0 <= c < W:
                        M[r, c] += F * wyv * wxv
    return M


def psf_centre(psf: np.ndarray):
    """The PSF's peak pixel (largest value, lowest row-major index on ties)."""
    p = int(np.argmax(np.asarray(psf, dtype=np.float64)))
    return divmod(p, psf.shape[1])


def convolve_psf(M: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """(B (*) M)(r, c) = sum M(r', c') B(ci + r - r', cj + c - c'), zero outside."""
    from scipy import fft as sfft
    from scipy.signal import fftconvolve
    ci, cj = psf_centre(psf)
    H, W = M.shape
    with sfft.set_workers(8):
        full = fftconvolve(M, np.asarray(psf, dtype=np.float64), mode="full")
    return full[ci:ci + H, cj:cj + W]


def refreshed_residual(dirty: np.ndarray, psf: np.ndarray, comps: np.ndarray,
                       alpha_b: float, omega_b: float, window_sigmas: float = 5.0) -> np.ndarray:
    """R = I_dirty - B (*) I_model (Sect. 2 step 3)."""
    D = np.asarray(dirty, dtype=np.float64)
    M = model_image(D.shape, comps, alpha_b, omega_b, window_sigmas)
    return D - convolve_psf(M, psf)
