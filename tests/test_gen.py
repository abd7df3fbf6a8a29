"""Sanity of the synthetic inputs (statistics, determinism); not parity."""
import math

import numpy as np
from scipy import integrate, special

from gen import configs as C
from gen import screens as S


def _vk_structure(r, r0, L0):
    # D(r) = 4 pi int_0^inf PSD(f) (1 - J0(2 pi f r)) f df, from the von Karman PSD
    f = lambda x: S.von_karman_psd(x, r0, L0) * (1 - special.j0(2 * np.pi * x * r)) * x
    v1, _ = integrate.quad(f, 0, 10.0 / r, limit=400)
    v2, _ = integrate.quad(f, 10.0 / r, np.inf, limit=400)
    return 4 * np.pi * (v1 + v2)


def test_screen_structure_function_matches_theory():
    scr = S.phase_screen(512, 0.1)
    for lag in (2, 5, 10):
        d = np.mean((scr[:, lag:] - scr[:, :-lag]) ** 2) * 0.5 + np.mean((scr[lag:, :] - scr[:-lag, :]) ** 2) * 0.5
        want = _vk_structure(lag * 0.1, C.SCREEN_R0_M, C.SCREEN_L0_M)
        assert abs(d / want - 1) < 0.15, (lag, d, want)
    # Kolmogorov limit at small separation
    r = 0.2
    assert abs(_vk_structure(r, 0.15, 1e6) / (6.88 * (r / 0.15) ** (5 / 3)) - 1) < 0.01


def test_screens_are_deterministic_and_seeded():
    a = S.ngs8m_opd(3)
    b = S.ngs8m_opd(3)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    assert not np.array_equal(S.phase_screen(64, 0.1, seed=1), S.phase_screen(64, 0.1, seed=2))
    assert np.array_equal(S.ngs8m_opd(2, frame0=1)[0], a[1])


def test_lgs_windows():
    o = S.lgs39m_opd(2, 6, pupil_n=800)
    assert o.shape == (2, 6, 800, 800)
    scr = S.screen_opd_m(2048, 4.875e-2).astype(np.float32)
    assert np.array_equal(o[1, 3], scr[300:1100, 301:1101])


def test_arrivals_rate():
    t = S.poisson_arrivals(2000.0, 5.0, 2000)
    assert abs(len(t) / 5.0 - 2000) < 5 * math.sqrt(2000 / 5.0)
    assert np.all(np.diff(t) > 0)
