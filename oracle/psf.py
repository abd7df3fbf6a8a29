"""Oracle science PSF and Strehl ratio (FP64, explicit DFT matrices).

Test infrastructure (see the package docstring).

Sec. 3 PSF block: the PSF is generated at the user's wavelength from the
closed-loop residual wavefront series, and the Strehl ratio is taken from
it; the integrated PSF of Sec. 5 is the sum over frames.  Reading O11: the
M x M transform is centred so that the on-axis direction falls on pixel
(M/2, M/2), and the PSF is normalised by (sum A)^2 so that the
diffraction-limited PSF has the value 1 on axis; the Strehl ratio is that
on-axis sample.
"""
from __future__ import annotations

import numpy as np

from . import geometry as G


def shifted_dft(M: int, n: int) -> np.ndarray:
    """W[u, x] = exp(-2 pi i (u - M/2) x / M) for x < n."""
    u = np.arange(M, dtype=np.float64)[:, None] - M / 2.0
    x = np.arange(n, dtype=np.float64)[None, :]
    return np.exp(-2j * np.pi * u * x / M)


def psf_frame(cfg, opd_m, W=None):
    """PSF of one residual OPD [N_p][N_p] (metres): |W e W^T|^2 / (sum A)^2."""
    A = G.pupil_mask(cfg.pupil_n, cfg.obstruction)
    e = A * np.exp(2j * np.pi * np.asarray(opd_m, dtype=np.float64) / cfg.wavelength_m)
    if W is None:
        W = shifted_dft(cfg.fft_m, cfg.pupil_n)
    F = W @ e @ W.T
    return (F.real ** 2 + F.imag ** 2) / (A.sum() ** 2)


def psf_accumulate(cfg, opd_frames):
    """Sum of the frame PSFs and the per-frame Strehl (on-axis sample)."""
    W = shifted_dft(cfg.fft_m, cfg.pupil_n)
    acc = np.zeros((cfg.fft_m, cfg.fft_m))
    sr = np.empty(len(opd_frames))
    c = cfg.fft_m // 2
    for i, opd in enumerate(opd_frames):
        P = psf_frame(cfg, opd, W)
        acc += P
        sr[i] = P[c, c]
    return acc, sr


def strehl_direct(cfg, opd_m):
    """|sum A e^{i phi}|^2 / (sum A)^2: the on-axis value with no transform."""
    A = G.pupil_mask(cfg.pupil_n, cfg.obstruction)
    e = A * np.exp(2j * np.pi * np.asarray(opd_m, dtype=np.float64) / cfg.wavelength_m)
    s = e.sum()
    return (s.real ** 2 + s.imag ** 2) / (A.sum() ** 2)


def encircled_energy(P, radii_px):
    """Fraction of sum P inside each radius (pixels) around the on-axis pixel (M/2, M/2) (Sec. 3 PSF
    block): pixels (v, u) with (u - M/2)^2 + (v - M/2)^2 <= r^2."""
    P = np.asarray(P, dtype=np.float64)
    M = P.shape[-1]
    c = M // 2
    d = np.arange(M, dtype=np.float64) - c
    d2 = d[None, :] ** 2 + d[:, None] ** 2
    tot = P.sum()
    return np.array([P[d2 <= float(r) ** 2].sum() / tot for r in radii_px])


def resample(P, scale):
    """PSF P put on the angular grid of another wavelength: Q[v, u] = P sampled bilinearly at
    (M/2 + (v - M/2) scale, M/2 + (u - M/2) scale), 0 where that point leaves the grid
    (reading O16; scale = lambda_ref / lambda of P)."""
    P = np.asarray(P, dtype=np.float64)
    M = P.shape[-1]
    c = M // 2
    g = c + (np.arange(M, dtype=np.float64) - c) * scale
    X, Y = np.meshgrid(g, g)
    ok = (X >= 0) & (Y >= 0) & (X <= M - 1) & (Y <= M - 1)
    ix = np.minimum(np.floor(np.where(ok, X, 0)).astype(np.int64), M - 2)
    iy = np.minimum(np.floor(np.where(ok, Y, 0)).astype(np.int64), M - 2)
    fx = np.where(ok, X, 0) - ix
    fy = np.where(ok, Y, 0) - iy
    Q = ((1 - fy) * ((1 - fx) * P[iy, ix] + fx * P[iy, ix + 1])
         + fy * ((1 - fx) * P[iy + 1, ix] + fx * P[iy + 1, ix + 1]))
    return np.where(ok, Q, 0.0)


def polychromatic(cfgs, weights, opd_frames):
    """Colour-weighted PSF on the grid of cfgs[0]'s wavelength: sum_i w_i resample(sum_f P_i,f)."""
    out = None
    for cfg, w in zip(cfgs, weights):
        acc, _ = psf_accumulate(cfg, opd_frames)
        q = w * resample(acc, cfgs[0].wavelength_m / cfg.wavelength_m)
        out = q if out is None else out + q
    return out


def airy_encircled_energy(r_px, pupil_n, fft_m):
    """Encircled energy of the PSF of an unobstructed circular pupil of pupil_n samples on an M grid:
    1 - J0(x)^2 - J1(x)^2, x = pi r pupil_n / M (the continuous-pupil closed form)."""
    from scipy.special import j0, j1
    x = np.pi * np.asarray(r_px, dtype=np.float64) * pupil_n / fft_m
    return 1.0 - j0(x) ** 2 - j1(x) ** 2
