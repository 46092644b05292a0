"""Seeded synthetic interferometric fields: the inputs of the minor cycle.

This module generates inputs only.  It implements the measurement model of
Sect. 2, Eq. (1) -- a dirty image is the true sky convolved with the PSF plus
noise -- and the sky as a finite sum of components (Eq. 2).  It holds none of
the deconvolution method's arithmetic: no fitting, no analytic Gaussian
convolution, no residual update.  Both the FP64 oracle and the HIP path are fed
from here, so a test can give both sides the identical arrays.

Every generator takes a seed and draws all randomness from
``numpy.random.default_rng(seed)``.  Images are row-major, ``img[row, col]``;
pixel centres sit at integer coordinates; ``x`` is the column, ``y`` the row.

The paper's workload (CASA-simulated L-band EVLA data of M31 with a six-hour
track and 32 channels over 1 GHz, Sect. 4) is not available; the Y-array PSF
below takes that instrument's character (three-armed array, L band, 32
channels, an earth-rotation track, uniform weighting) and the sky is a seeded
mix of point sources and circular Gaussians.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))  # 2.35482...
_FFT_WORKERS = 8


@dataclasses.dataclass
class Field:
    """One synthetic field and the run parameters it is deconvolved with."""
    name: str
    dirty: np.ndarray          # float32 [H, W]
    psf: np.ndarray            # float32 [Hp, Wp], peak 1
    gain: float
    threshold: float
    max_iter: int
    max_active: int
    points: np.ndarray         # float64 [P, 3]: (x, y, flux)        sky-plane truth
    gaussians: np.ndarray      # float64 [G, 4]: (x, y, sigma, peak) sky-plane truth
    noise_sigma: float
    psf_fwhm: float | None = None   # set for analytic Gaussian PSFs
    seed: int = 0

    @property
    def shape(self):
        return self.dirty.shape


# ----------------------------------------------------------------------------
# Sky rendering (Eq. 2: the sky is a sum of components)
# ----------------------------------------------------------------------------

def render_sky(H: int, W: int, points: np.ndarray, gaussians: np.ndarray) -> np.ndarray:
    """Sky image in FP64.  Points sit on integer pixels and carry their flux in
    that pixel; Gaussians are point-sampled at pixel centres out to 8 sigma."""
    sky = np.zeros((H, W), dtype=np.float64)
    for x, y, f in points:
        sky[int(y), int(x)] += f
    for x, y, sig, peak in gaussians:
        h = int(math.ceil(8.0 * sig))
        r0, r1 = max(0, int(math.floor(y)) - h), min(H - 1, int(math.floor(y)) + h + 1)
        c0, c1 = max(0, int(math.floor(x)) - h), min(W - 1, int(math.floor(x)) + h + 1)
        rr = np.arange(r0, r1 + 1, dtype=np.float64)[:, None] - y
        cc = np.arange(c0, c1 + 1, dtype=np.float64)[None, :] - x
        sky[r0:r1 + 1, c0:c1 + 1] += peak * np.exp(-(rr * rr + cc * cc) / (2.0 * sig * sig))
    return sky


def gaussian_psf(n: int, fwhm: float) -> np.ndarray:
    """An n x n circular Gaussian PSF with peak exactly 1 at pixel (n//2, n//2)."""
    sig = fwhm / FWHM_PER_SIGMA
    c = n // 2
    r = np.arange(n, dtype=np.float64) - c
    return np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * sig * sig))


def convolve_linear(sky: np.ndarray, psf: np.ndarray, centre: tuple[int, int]) -> np.ndarray:
    """out[i, j] = sum_{k,l} sky[k, l] * psf[ci + i - k, cj + j - l]  (zero outside psf).

    A plain linear convolution by zero-padded FFT in FP64; ``centre`` is the
    PSF's peak pixel (ci, cj)."""
    H, W = sky.shape
    Hp, Wp = psf.shape
    ci, cj = centre
    fh, fw = H + Hp - 1, W + Wp - 1
    sh, sw = sfft.next_fast_len(fh, real=True), sfft.next_fast_len(fw, real=True)
    full = sfft.irfft2(sfft.rfft2(sky, s=(sh, sw), workers=_FFT_WORKERS)
                       * sfft.rfft2(psf, s=(sh, sw), workers=_FFT_WORKERS),
                       s=(sh, sw), workers=_FFT_WORKERS)
    return full[ci:ci + H, cj:cj + W].copy()


# ----------------------------------------------------------------------------
# Y-array PSF (uniform weighting)
# ----------------------------------------------------------------------------

C_LIGHT = 299_792_458.0


def yarray_enu(arm_len_m: float = 5200.0, per_arm: int = 9, power: float = 1.716,
               arm_az_deg=(5.0, 125.0, 245.0)) -> np.ndarray:
    """Antenna positions (east, north) in metres of a three-armed Y array with
    power-law spacing along each arm (27 antennas by default)."""
    pos = []
    for az in arm_az_deg:
        a = math.radians(az)
        for k in range(1, per_arm + 1):
            r = arm_len_m * (k / per_arm) ** power
            pos.append((r * math.sin(a), r * math.cos(a)))
    return np.asarray(pos, dtype=np.float64)


def yarray_uv(lat_deg: float = 34.0, dec_deg: float = 40.0, ha_hours: float = 4.0,
              dt_s: float = 60.0, f_lo: float = 1.0e9, f_hi: float = 2.0e9,
              n_chan: int = 32, **enu_kw) -> tuple[np.ndarray, np.ndarray]:
    """(u, v) in wavelengths for every baseline, time sample and channel of an
    earth-rotation track from -ha_hours to +ha_hours (both conjugates)."""
    enu = yarray_enu(**enu_kw)
    lat, dec = math.radians(lat_deg), math.radians(dec_deg)
    # local (east, north, up=0) -> equatorial (X, Y, Z)
    X = -math.sin(lat) * enu[:, 1]
    Y = enu[:, 0]
    Z = math.cos(lat) * enu[:, 1]
    i, j = np.triu_indices(len(enu), k=1)
    bx, by, bz = X[j] - X[i], Y[j] - Y[i], Z[j] - Z[i]
    n_t = int(round(2 * ha_hours * 3600.0 / dt_s)) + 1
    ha = np.linspace(-ha_hours, ha_hours, n_t) * (math.pi / 12.0)
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    u_m = sh * bx + ch * by
    v_m = -math.sin(dec) * ch * bx + math.sin(dec) * sh * by + math.cos(dec) * bz
    freqs = (f_lo + (np.arange(n_chan) + 0.5) * (f_hi - f_lo) / n_chan)
    lam_inv = freqs / C_LIGHT
    u = (u_m.ravel()[:, None] * lam_inv[None, :]).ravel()
    v = (v_m.ravel()[:, None] * lam_inv[None, :]).ravel()
    return np.concatenate([u, -u]), np.concatenate([v, -v])


def yarray_uv_grid(grid_n: int, cell_frac: float = 0.30, taper: float = 0.45,
                   **uv_kw) -> np.ndarray:
    """Uniformly weighted, Gaussian-tapered uv sampling grid (FFT layout, origin
    at [0, 0]).

    Each sampled cell gets weight 1 (uniform weighting = 1 / samples per cell),
    then an outer Gaussian taper exp(-|u|^2 / (2 (taper * u_max)^2)).  Uniform
    weighting alone gives an Airy-like ~12 % first sidelobe; the taper brings
    the peak sidelobe to ~4 % with a main-lobe FWHM of ~3.5 px.
    ``cell_frac`` is the largest |u| or |v| as a fraction of the grid size, which
    sets the pixel scale."""
    u, v = yarray_uv(**uv_kw)
    umax = max(np.abs(u).max(), np.abs(v).max())
    du = umax / (cell_frac * grid_n)
    iu = np.rint(u / du).astype(np.int64) % grid_n
    iv = np.rint(v / du).astype(np.int64) % grid_n
    grid = np.zeros((grid_n, grid_n), dtype=np.float64)
    grid[iv, iu] = 1.0
    # enforce Hermitian symmetry on the grid so the PSF is real
    grid = np.maximum(grid, np.roll(grid[::-1, ::-1], 1, axis=(0, 1)))
    k = np.fft.fftfreq(grid_n) * grid_n
    st = taper * cell_frac * grid_n
    tap = np.exp(-(k * k) / (2.0 * st * st))
    grid *= tap[:, None]
    grid *= tap[None, :]
    return grid


def psf_from_grid(grid: np.ndarray) -> np.ndarray:
    """Periodic PSF (origin at [0, 0]) of a weighted uv grid, peak normalised to 1."""
    psf = sfft.ifft2(grid, workers=_FFT_WORKERS).real
    return psf / psf[0, 0]


def psf_stats(psf_centred: np.ndarray) -> dict:
    """Main-lobe FWHM (px, from the half-power area) and the largest |sidelobe|
    outside the main lobe, for a PSF whose peak is at the array centre."""
    n0, n1 = psf_centred.shape
    c0, c1 = n0 // 2, n1 // 2
    # main lobe: 4-connected region around the peak with psf > 0
    from scipy import ndimage
    lab, _ = ndimage.label(psf_centred > 0.0)
    main = lab == lab[c0, c1]
    half = (psf_centred >= 0.5) & main
    fwhm = 2.0 * math.sqrt(half.sum() / math.pi)
    side = np.abs(psf_centred[~main]).max()
    return {"fwhm_px": fwhm, "peak_sidelobe": float(side),
            "min": float(psf_centred.min())}


# ----------------------------------------------------------------------------
# Sky draws
# ----------------------------------------------------------------------------

def powerlaw_flux(rng, n: int, s_min: float, s_max: float) -> np.ndarray:
    """Fluxes with dN/dS ~ S^-1.5 on [s_min, s_max] by inverse CDF."""
    u = rng.random(n)
    a, b = s_min ** -0.5, s_max ** -0.5
    return (a + u * (b - a)) ** -2.0


def _draw_sky(rng, H, W, n_points, n_gauss, sigma_lo, sigma_hi, flux_lo, flux_hi,
              powerlaw, edge=8):
    px = rng.integers(edge, W - edge, size=n_points)
    py = rng.integers(edge, H - edge, size=n_points)
    if powerlaw:
        pf = powerlaw_flux(rng, n_points, flux_lo, flux_hi)
    else:
        pf = rng.uniform(flux_lo, flux_hi, size=n_points)
    points = np.stack([px, py, pf], axis=1).astype(np.float64)
    gs = []
    for _ in range(n_gauss):
        sig = rng.uniform(sigma_lo, sigma_hi)
        m = min(3.0 * sig, 0.45 * min(H, W))
        gx = rng.uniform(m, W - 1 - m)
        gy = rng.uniform(m, H - 1 - m)
        gs.append((gx, gy, sig, rng.uniform(0.05, 0.5)))
    gaussians = np.asarray(gs, dtype=np.float64).reshape(-1, 4)
    return points, gaussians


# ----------------------------------------------------------------------------
# The workloads
# ----------------------------------------------------------------------------

def make_c128(seed: int = 0) -> Field:
    """128 x 128: 5 points (flux U[0.1, 1] on integer pixels in [8, 119]) and 3
    circular Gaussians (sigma U[2, 8] px, sky peak U[0.05, 0.5]), convolved with
    an exact Gaussian PSF of FWHM 3 px, plus N(0, 1e-3) white noise.  Run: gain
    0.1, threshold 5e-3, at most 200 iterations, active set at most 5."""
    rng = np.random.default_rng(seed)
    H = W = 128
    px = rng.integers(8, 120, size=5)
    py = rng.integers(8, 120, size=5)
    pf = rng.uniform(0.1, 1.0, size=5)
    points = np.stack([px, py, pf], axis=1).astype(np.float64)
    gs = []
    for _ in range(3):
        sig = rng.uniform(2.0, 8.0)
        gx = rng.uniform(3 * sig, 127 - 3 * sig)
        gy = rng.uniform(3 * sig, 127 - 3 * sig)
        gs.append((gx, gy, sig, rng.uniform(0.05, 0.5)))
    gaussians = np.asarray(gs, dtype=np.float64)
    psf = gaussian_psf(128, 3.0)
    sky = render_sky(H, W, points, gaussians)
    dirty = convolve_linear(sky, psf, (64, 64)) + rng.normal(0.0, 1e-3, size=(H, W))
    return Field("c128", dirty.astype(np.float32), psf.astype(np.float32), 0.1, 5e-3, 200, 5,
                 points, gaussians, 1e-3, psf_fwhm=3.0, seed=seed)


def make_evla(n: int, seed: int, n_points: int, n_gauss: int, sigma_hi: float,
              max_iter: int, max_active: int, psf_crop: int = 256,
              noise: float = 1e-4, name: str | None = None) -> Field:
    """An n x n field with the Y-array PSF gridded on 2n x 2n, a power-law point
    population (flux 1e-3..1, dN/dS ~ S^-1.5) and circular Gaussians with sigma
    U[2, sigma_hi] px and sky peak U[0.05, 0.5]; N(0, noise) white noise.  The
    dirty image is the periodic convolution on the 2n grid (the PSF of a gridded
    uv coverage is itself periodic on that grid), cropped to n x n."""
    rng = np.random.default_rng(seed)
    g = 2 * n
    grid = yarray_uv_grid(g)
    points, gaussians = _draw_sky(rng, n, n, n_points, n_gauss, 2.0, sigma_hi, 1e-3, 1.0,
                                  powerlaw=True)
    sky = render_sky(n, n, points, gaussians)
    norm = sfft.ifft2(grid, workers=_FFT_WORKERS).real[0, 0]
    # dirty = sky (*) psf  with psf = ifft(grid)/norm  =>  ifft(fft(sky) * grid)/norm
    half = grid[:, : g // 2 + 1]
    spec = sfft.rfft2(sky, s=(g, g), workers=_FFT_WORKERS)
    spec *= half
    dirty = sfft.irfft2(spec, s=(g, g), workers=_FFT_WORKERS)[:n, :n] / norm
    del spec
    dirty += rng.normal(0.0, noise, size=(n, n))
    psf_full = psf_from_grid(grid)
    psf = np.fft.fftshift(psf_full)
    c = g // 2
    h = psf_crop // 2
    psf = psf[c - h:c + h, c - h:c + h]
    return Field(name or f"c{n}", dirty.astype(np.float32), psf.astype(np.float32), 0.1, 0.0,
                 max_iter, max_active, points, gaussians, noise, seed=seed)


def make_c1024(seed: int = 1000) -> Field:
    """1024 x 1024: 200 points + 40 Gaussians (sigma U[2, 40] px); 5000
    iterations, threshold 0, gain 0.1, active set at most 5."""
    return make_evla(1024, seed, 200, 40, 40.0, 5000, 5, name="c1024")


def make_c4096(seed: int = 4096) -> Field:
    """4096 x 4096: 2000 points + 300 Gaussians (sigma U[2, 120] px); 20000
    iterations, threshold 0, gain 0.1, active set at most 10."""
    return make_evla(4096, seed, 2000, 300, 120.0, 20000, 10, name="c4096")


def batch_sizes(seed: int = 64, n_fields: int = 64) -> list[int]:
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice([256, 512, 1024, 2048], size=n_fields)]


def make_batch_field(n: int, seed: int, max_iter: int = 5000) -> Field:
    """One field of the batched workload: the sky of the 1024 x 1024 generator
    with counts scaled by area, sigma U[2, min(40, n/16)], and an exact Gaussian
    PSF of FWHM U[2.5, 6] px; N(0, 1e-4) noise."""
    rng = np.random.default_rng(seed)
    scale = (n / 1024.0) ** 2
    n_pts = max(1, int(round(200 * scale)))
    n_g = max(1, int(round(40 * scale)))
    fwhm = rng.uniform(2.5, 6.0)
    points, gaussians = _draw_sky(rng, n, n, n_pts, n_g, 2.0, min(40.0, n / 16.0), 1e-3, 1.0,
                                  powerlaw=True)
    sky = render_sky(n, n, points, gaussians)
    pn = 64
    psf = gaussian_psf(pn, fwhm)
    dirty = convolve_linear(sky, psf, (pn // 2, pn // 2)) + rng.normal(0.0, 1e-4, size=(n, n))
    return Field(f"b{n}", dirty.astype(np.float32), psf.astype(np.float32), 0.1, 0.0, max_iter, 5,
                 points, gaussians, 1e-4, psf_fwhm=fwhm, seed=seed)


def make_batch(seed: int = 64, n_fields: int = 64, max_iter: int = 5000) -> list[Field]:
    return [make_batch_field(n, 6400 + i, max_iter) for i, n in
            enumerate(batch_sizes(seed, n_fields))]


def isolated_gaussian(H: int, W: int, amp: float, x: float, y: float, sigma: float) -> np.ndarray:
    """A single point-sampled Gaussian image (FP64)."""
    rr = np.arange(H, dtype=np.float64)[:, None] - y
    cc = np.arange(W, dtype=np.float64)[None, :] - x
    return amp * np.exp(-(rr * rr + cc * cc) / (2.0 * sigma * sigma))


def random_image(H: int, W: int, seed: int, dist: str = "normal") -> np.ndarray:
    """Seeded float32 test image for kernel-level checks."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        return rng.normal(size=(H, W)).astype(np.float32)
    if dist == "int":
        return rng.integers(-8, 9, size=(H, W)).astype(np.float32)
    raise ValueError(dist)
