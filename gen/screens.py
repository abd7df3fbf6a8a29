"""Seeded synthetic inputs: phase screens, OPD stacks, DM coefficients, arrivals.

Nothing here is part of the measured sensor path.  Phase screens follow
the block "atmospheric layers generation" of paper Sec. 3: a screen is the
inverse FFT of white noise shaped by the square root of the von Karman
phase power spectrum.  Everything is FP64 and converted to FP32 OPD in
metres, the form both the oracle and the GPU path consume.
"""
from __future__ import annotations

import functools

import numpy as np

from . import configs as C


def von_karman_psd(f, r0_m, L0_m):
    """Phase PSD (rad^2 m^2) at the wavelength r0 is quoted at."""
    return 0.0229 * r0_m ** (-5.0 / 3.0) * (f * f + 1.0 / (L0_m * L0_m)) ** (-11.0 / 6.0)


@functools.lru_cache(maxsize=4)
def phase_screen(n: int, dx_m: float, r0_m: float = C.SCREEN_R0_M, L0_m: float = C.SCREEN_L0_M,
                 seed: int = C.SCREEN_SEED) -> np.ndarray:
    """n x n von Karman phase screen in radians at 0.5 um (FP64, read-only)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fx = np.fft.fftfreq(n, d=dx_m)
    f = np.hypot(fx[None, :], fx[:, None])
    df = 1.0 / (n * dx_m)
    amp = np.sqrt(von_karman_psd(f, r0_m, L0_m)) * df
    amp[0, 0] = 0.0
    noise = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    scr = np.real(np.fft.ifft2(noise * amp)) * (n * n)
    scr.setflags(write=False)
    return scr


def screen_opd_m(n: int, dx_m: float, seed: int = C.SCREEN_SEED) -> np.ndarray:
    """The screen as OPD in metres (FP64)."""
    return phase_screen(n, dx_m, seed=seed) * (C.SCREEN_LAMBDA0_M / (2.0 * np.pi))


def ngs8m_opd(n_frames: int, frame0: int = 0, seed: int = C.SCREEN_SEED) -> np.ndarray:
    """8 m workload: [n_frames][80][80] FP32 OPD; frame t is the window at
    (row t // 432, col t % 432) of a 512^2 screen at 0.1 m/px."""
    scr = screen_opd_m(512, 0.1, seed)
    out = np.empty((n_frames, 80, 80), np.float32)
    for i in range(n_frames):
        t = frame0 + i
        r0, c0 = (t // 432) % 432, t % 432
        out[i] = scr[r0:r0 + 80, c0:c0 + 80]
    return out


def lgs39m_opd(n_frames: int, n_wfs: int = 6, frame0: int = 0, seed: int = C.SCREEN_SEED,
               pupil_n: int = 800) -> np.ndarray:
    """39 m workload: [n_frames][n_wfs][pupil_n][pupil_n] FP32 OPD; sensor w looks through
    the window whose origin is row 100*w, column 100*w + t of a 2048^2 screen."""
    scr = screen_opd_m(2048, 4.875e-2, seed)
    out = np.empty((n_frames, n_wfs, pupil_n, pupil_n), np.float32)
    for i in range(n_frames):
        t = (frame0 + i) % (2048 - pupil_n - 100 * (n_wfs - 1) + 1)
        for w in range(n_wfs):
            out[i, w] = scr[100 * w:100 * w + pupil_n, 100 * w + t:100 * w + t + pupil_n]
    return out


def dm_coefficients(n_act: int, seed: int, rms_m: float = C.DM_COEF_RMS_M) -> np.ndarray:
    """Random DM actuator commands (OPD metres), FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n_act) * rms_m


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate_hz * duration_s * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    return t[t < duration_s]


def random_opd(shape, rms_m: float, seed: int) -> np.ndarray:
    """White OPD (FP32) for edge-case and stress inputs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(shape) * rms_m).astype(np.float32)
