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
