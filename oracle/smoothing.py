"""FP64 oracle of the smoothing initial values -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP library.

What it computes (Sect. 2, step 1 of the Asp-Clean loop; Sect. 3, the
paragraph on initial values; the conclusion): the residual is smoothed with a
few Gaussian beams, the peak over all smoothed images is found, and the
Gaussian of that peak -- its place, its width and an amplitude -- is the
initial guess of the new component.  Sect. 3 then switches between this
smoothing method and the simple method (residual peak, main-lobe width) by the
area of the last fitted component against the area of its initial guess.

Readings where the paper is silent (each listed in the design notes):

* Trial widths: sigma_j = omega_b * 2**j, j = 0 .. n_scales - 1, kept while
  sigma_j <= s_max (the fit's upper width bound); sigma_0 = omega_b is the beam
  itself, so a PSF-sized feature is matched at j = 0.
* Smoothing kernel of width sigma: K(dy, dx) = exp(-(dx^2 + dy^2) / (2 sigma^2))
  on the square window |dx|, |dy| <= h(sigma) = max(3, ceil(c_w sigma)), the
  window a component of that width is evaluated on.  The smoothed image at
  pixel p is C(p) = sum over the window around p, clipped to the image, of
  K(q - p) R(q) (the residual is zero outside the image).
* Cross-scale comparison: the smoothing beams have peak 1 (as the PSF has),
  and the peak among the smoothed images is the largest |C(p)| over all
  scales, compared as they are (norm "peak", the default).  The alternative
  reading (norm "l2") divides by the kernel's norm over the clipped window,
  S(p) = C(p) / sqrt(N(p)), N(p) = sum of K(q - p)^2 over that window; then
  S(p)^2 is the drop in the squared residual when the least-squares multiple
  C(p)/N(p) of that Gaussian is subtracted (a matched filter).
* The peak is the largest |S| over all (j, p); ties go to the smallest j, then
  to the smallest row-major p.  Start values: the least-squares amplitude
  C(p)/N(p) of that Gaussian at that pixel, centre p, width sigma_j
  (convolved space).
* The switch (Sect. 3): the simple method is used in an iteration when, in
  the previous iteration, the area of the fitted new component was below 5 %
  of the area of its initial guess; otherwise the smoothing method.  Areas are
  those of the convolved-space Gaussians, pi s^2 (alternative reading: the
  deconvolved pi (s^2 - omega_b^2)).  The first iteration smooths.

Two evaluations of C and N: ``direct`` sums over the window pixel by pixel
(the definition), ``fft`` takes the same zero-padded convolution through
scipy's FFT (a library primitive; the kernel is symmetric, so convolution and
correlation agree).  The tests pin both against each other and against brute
force least squares.
"""
from __future__ import annotations

import math

import numpy as np

AREA_FRACTION = 0.05


def halfwidth(s: float, window_sigmas: float = 5.0) -> int:
    """Window half-width of a Gaussian of width s: max(3, ceil(c_w s))."""
    h = math.ceil(window_sigmas * s)
    return int(max(3, h))


def widths(omega_b: float, n_scales: int, s_max: float) -> list[float]:
    """The trial widths omega_b * 2**j that do not exceed s_max (at least omega_b)."""
    out = []
    for j in range(max(1, int(n_scales))):
        s = omega_b * float(2 ** j)
        if j > 0 and s > s_max:
            break
        out.append(s)
    return out


def kernel(sigma: float, window_sigmas: float = 5.0) -> np.ndarray:
    """The (2h+1) x (2h+1) smoothing Gaussian, peak 1 at the centre."""
    h = halfwidth(sigma, window_sigmas)
    d = np.arange(-h, h + 1, dtype=np.float64)
    q = d[:, None] ** 2 + d[None, :] ** 2
    return np.exp(-q / (2.0 * sigma * sigma))


def _conv_fft(img: np.ndarray, K: np.ndarray) -> np.ndarray:
    from scipy import fft as sfft
    from scipy.signal import fftconvolve
    h = K.shape[0] // 2
    H, W = img.shape
    with sfft.set_workers(8):
        full = fftconvolve(img, K, mode="full")
    return full[h:h + H, h:h + W]


def _conv_direct(img: np.ndarray, K: np.ndarray) -> np.ndarray:
    """out(p) = sum over the clipped window of K(q - p) img(q), offset by offset."""
    h = K.shape[0] // 2
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.float64)
    for dy in range(-h, h + 1):
        r0, r1 = max(0, -dy), min(H, H - dy)      # output rows whose r + dy is inside
        if r0 >= r1:
            continue
        for dx in range(-h, h + 1):
            c0, c1 = max(0, -dx), min(W, W - dx)
            if c0 >= c1:
                continue
            out[r0:r1, c0:c1] += K[dy + h, dx + h] * img[r0 + dy:r1 + dy, c0 + dx:c1 + dx]
    return out


def smoothed(R: np.ndarray, sigma: float, window_sigmas: float = 5.0,
             method: str = "fft", need_norm: bool = True):
    """(C, N): the residual smoothed with the Gaussian of width sigma, and the
    squared norm of the clipped kernel at every pixel (None unless need_norm)."""
    R = np.asarray(R, dtype=np.float64)
    K = kernel(sigma, window_sigmas)
    conv = _conv_fft if method == "fft" else _conv_direct
    return conv(R, K), (conv(np.ones_like(R), K * K) if need_norm else None)


NORMS = ("peak", "l2")


def scores(R: np.ndarray, omega_b: float, n_scales: int, s_max: float,
           window_sigmas: float = 5.0, method: str = "fft", norm: str = "peak"):
    """Per trial width: (sigma, C, N, S), S = C (norm "peak") or C / sqrt(N)
    (norm "l2")."""
    if norm not in NORMS:
        raise ValueError(norm)
    out = []
    for s in widths(omega_b, n_scales, s_max):
        C, N = smoothed(R, s, window_sigmas, method, need_norm=(norm == "l2"))
        out.append((s, C, N, C if norm == "peak" else C / np.sqrt(N)))
    return out


def auto_method(shape, omega_b: float, n_scales: int, s_max: float,
                window_sigmas: float = 5.0) -> str:
    """The definition's direct sums while they are cheap, else the FFT."""
    n = shape[0] * shape[1]
    work = sum((2 * halfwidth(s, window_sigmas) + 1) ** 2 for s in widths(omega_b, n_scales, s_max))
    return "direct" if n * work <= 3e7 else "fft"


def best(R: np.ndarray, omega_b: float, n_scales: int, s_max: float,
         window_sigmas: float = 5.0, method: str | None = None, norm: str = "peak") -> dict:
    """The peak over all smoothed images and the start values it gives."""
    R = np.asarray(R, dtype=np.float64)
    if method is None:
        method = auto_method(R.shape, omega_b, n_scales, s_max, window_sigmas)
    sc = scores(R, omega_b, n_scales, s_max, window_sigmas, method, norm)
    stack = np.stack([np.abs(S).ravel() for (_, _, _, S) in sc])
    flat = int(np.argmax(stack))            # first maximum: smallest j, then smallest p
    j, p = divmod(flat, R.size)
    s, C, N, S = sc[j]
    r, c = divmod(p, R.shape[1])
    c_ = float(C.ravel()[p])
    n_ = float(N.ravel()[p]) if N is not None else score_at(R, s, p, window_sigmas)[1]
    return {"scale": j, "idx": p, "sigma": s, "score": float(S.ravel()[p]), "corr": c_,
            "norm2": n_, "start": np.array([c_ / n_, float(c), float(r), s]),
            "maps": sc, "method": method}


def score_at(R: np.ndarray, sigma: float, idx: int, window_sigmas: float = 5.0,
             norm: str = "peak"):
    """(C, N, S) at one pixel by the direct sum over its window."""
    R = np.asarray(R, dtype=np.float64)
    H, W = R.shape
    r, c = divmod(int(idx), W)
    h = halfwidth(sigma, window_sigmas)
    r0, r1, c0, c1 = max(0, r - h), min(H - 1, r + h), max(0, c - h), min(W - 1, c + h)
    dy = np.arange(r0, r1 + 1, dtype=np.float64)[:, None] - r
    dx = np.arange(c0, c1 + 1, dtype=np.float64)[None, :] - c
    K = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
    C = float(np.sum(K * R[r0:r1 + 1, c0:c1 + 1]))
    N = float(np.sum(K * K))
    return C, N, (C if norm == "peak" else C / math.sqrt(N))


def simple_next(s_fit: float, s0: float, omega_b: float, deconvolved: bool = False) -> bool:
    """Sect. 3's switch: the simple method is due when the fitted new component's
    area is below 5 % of the area of its initial guess."""
    if deconvolved:
        return (s_fit * s_fit - omega_b * omega_b) < AREA_FRACTION * (s0 * s0 - omega_b * omega_b)
    return s_fit * s_fit < AREA_FRACTION * (s0 * s0)
