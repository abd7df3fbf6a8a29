"""Oracle geometry: pupil, sub-apertures, plate scales, sodium kernel (FP64).

Test infrastructure (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

ARCSEC = math.pi / (180.0 * 3600.0)


def pupil_mask(pupil_n: int, obstruction: float) -> np.ndarray:
    """Binary pupil A (Sec. 2 pupil sampling; reading O1).

    Pixel j has its centre at (j + 1/2 - N/2) pixels from the pupil centre;
    the pixel is lit iff eps*N/2 <= r <= N/2.  Distances are compared in
    squared pixel units, which is exact for half-integer coordinates.
    """
    a = np.arange(pupil_n, dtype=np.float64) + 0.5 - pupil_n / 2.0
    r2 = a[None, :] ** 2 + a[:, None] ** 2
    outer = (pupil_n / 2.0) ** 2
    inner = (obstruction * pupil_n / 2.0) ** 2
    return ((r2 <= outer) & (r2 >= inner)).astype(np.float64)


def subap_table(cfg):
    """Valid sub-apertures (Sec. 4: "the WF is split into sub-apertures"; reading O2).

    Returns (valid_idx, illum): the row-major indices a*n_subap + b of the
    valid sub-apertures and their illuminated fractions.
    """
    A = pupil_mask(cfg.pupil_n, cfg.obstruction)
    n = cfg.pupil_n // cfg.n_subap
    counts = A.reshape(cfg.n_subap, n, cfg.n_subap, n).sum(axis=(1, 3)).ravel()
    frac = counts / float(n * n)
    valid = np.nonzero(frac >= cfg.min_illum)[0]
    return valid.astype(np.int64), frac[valid]


def subap_centres_m(cfg, valid_idx):
    """Sub-aperture centres (x, y) in metres: the mean of its pixel centres."""
    n = cfg.pupil_n // cfg.n_subap
    a = valid_idx // cfg.n_subap
    b = valid_idx % cfg.n_subap
    xs = ((b + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    ys = ((a + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    return xs, ys


def fft_pixel_rad(cfg) -> float:
    """Angular size of one spot-FFT pixel, lambda / (fft_n dx) (reading O4)."""
    return cfg.wavelength_m / (cfg.fft_n * cfg.pupil_dx_m)


def det_pixel_rad(cfg) -> float:
    """Angular size of one detector pixel: conv_n / det_n FFT pixels (reading O4)."""
    return fft_pixel_rad(cfg) * cfg.conv_n / cfg.det_n


def elongation_params(cfg, launch_xy, valid_idx):
    """Per sub-aperture Gaussian parameters (Sec. 4 LGS module; reading O5).

    Returns (sigma_par, sigma_perp, psi) in conv-grid pixels and radians.
    The long axis points from the launcher to the sub-aperture; its FWHM
    adds the elongation (linear in distance, capped at elong_max_arcsec
    across the full diameter, or the geometric d*fwhm/H^2 when the cap is
    <= 0) in quadrature to the laser spot size.
    """
    xs, ys = subap_centres_m(cfg, valid_idx)
    lx, ly = launch_xy
    dxv = xs - lx
    dyv = ys - ly
    d = np.hypot(dxv, dyv)
    psi = np.arctan2(dyv, dxv)
    if cfg.elong_max_arcsec > 0:
        el = cfg.elong_max_arcsec * d / cfg.diameter_m
    else:
        el = d * cfg.na_fwhm_m / (cfg.na_height_m ** 2) / ARCSEC
    f_par = np.sqrt(el * el + cfg.spot_fwhm_arcsec ** 2)
    f_perp = np.full_like(f_par, cfg.spot_fwhm_arcsec)
    px_as = fft_pixel_rad(cfg) / ARCSEC
    to_sigma = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    return f_par * to_sigma / px_as, f_perp * to_sigma / px_as, psi


def sodium_kernel(N: int, sigma_par: float, sigma_perp: float, psi: float, reach: int = 3):
    """Periodised, normalised elongated Gaussian k on an N x N circular grid (reading O5).

    k[i, j] sums g over every lattice point (tx, ty) with tx = j, ty = i
    (mod N) and |tx|, |ty| <= reach*N.  The lattice window is symmetric, so
    k is exactly point-symmetric about (0, 0) and its DFT is real.
    Index i is the row (y), j the column (x).
    """
    c, s = math.cos(psi), math.sin(psi)
    t = np.arange(-reach * N, reach * N + 1, dtype=np.float64)
    tx = t[None, :]
    ty = t[:, None]
    along = tx * c + ty * s
    across = -tx * s + ty * c
    g = np.exp(-0.5 * (along * along / (sigma_par * sigma_par)
                       + across * across / (sigma_perp * sigma_perp)))
    k = np.zeros((N, N))
    idx = np.mod(t.astype(np.int64), N)
    np.add.at(k, (idx[:, None], idx[None, :]), g)
    return k / k.sum()


def dft_matrix(N: int) -> np.ndarray:
    """Plain DFT matrix, F[u, j] = exp(-2 pi i u j / N)."""
    u = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(u, u) / N)


def kernel_spectrum(k: np.ndarray) -> np.ndarray:
    """K^ = DFT2(k) (complex; real up to rounding for the symmetric kernels)."""
    F = dft_matrix(k.shape[0])
    return F @ k @ F.T
