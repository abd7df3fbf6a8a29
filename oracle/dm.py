"""Oracle deformable mirrors and residual OPD (FP64).

Test infrastructure (see the package docstring).

Sec. 3 closed-loop block: the residual phase is the open-loop wavefront
minus the DM.  Sec. 2: ~5000 modes on the ground DM and ~1400 and ~1800
on the two post-focal DMs with 1 m pitch; Sec. 3 influence-function
block: the tool computes influence functions analytically when none are
supplied.  Reading O12: Gaussian influence functions with coupling 0.3 at
one pitch on 64x64-pixel patches, actuators on a square grid inside the
metapupil of a 60 arcsec field radius, integer-pixel footprint shifts.
"""
from __future__ import annotations

import math

import numpy as np

ARCSEC = math.pi / (180.0 * 3600.0)


def metapupil_radius_px(pupil_n, dx_m, alt_m, field_radius_arcsec):
    return pupil_n / 2.0 + alt_m * field_radius_arcsec * ARCSEC / dx_m


def surface_size(pupil_n, dx_m, alt_m, field_radius_arcsec):
    """Side of the square DM surface array: 2 * ceil(metapupil radius)."""
    return 2 * int(math.ceil(metapupil_radius_px(pupil_n, dx_m, alt_m, field_radius_arcsec) - 1e-9))


def actuators(pupil_n, dx_m, alt_m, pitch_px, field_radius_arcsec):
    """Actuator positions (px from the DM centre) on a square grid within the metapupil."""
    R = metapupil_radius_px(pupil_n, dx_m, alt_m, field_radius_arcsec)
    m = int(math.floor(R / pitch_px))
    i = np.arange(-m, m + 1)
    X, Y = np.meshgrid(i * pitch_px, i * pitch_px)
    keep = X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2 <= R * R
    return np.stack([X[keep], Y[keep]], axis=1).astype(np.float64)   # (x, y), row-major in y


def influence_sigma(pitch_px, coupling):
    """Gaussian width with IF(pitch) = coupling."""
    return pitch_px / math.sqrt(2.0 * math.log(1.0 / coupling))


def dm_surface(size, act_xy, coefs, pitch_px, coupling=0.3, patch=64):
    """Sum_k c_k IF_k on a size x size grid whose centre is the DM centre.

    IF_k(p) = exp(-|p - a_k|^2 / (2 sigma^2)) on the patch x patch pixels
    nearest to a_k; pixel centres at (j + 1/2 - size/2).
    """
    sig = influence_sigma(pitch_px, coupling)
    surf = np.zeros((size, size))
    h = patch // 2
    for (ax, ay), c in zip(act_xy, coefs):
        cx = int(round(size / 2 + ax))
        cy = int(round(size / 2 + ay))
        j0, j1 = max(cx - h, 0), min(cx + h, size)
        i0, i1 = max(cy - h, 0), min(cy + h, size)
        xs = np.arange(j0, j1) + 0.5 - size / 2.0 - ax
        ys = np.arange(i0, i1) + 0.5 - size / 2.0 - ay
        surf[i0:i1, j0:j1] += c * np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * sig * sig))
    return surf


def footprint_shift_px(alt_m, theta_arcsec, dx_m):
    """Integer shift of a star's pupil footprint on a layer at alt_m: round(h theta / dx)."""
    return int(math.floor(alt_m * theta_arcsec * ARCSEC / dx_m + 0.5))


def residual_opd(screen, scr_origin, surfaces, origins, pupil_n):
    """screen[window] - sum_d surface_d[window_d]; origins are (row, col) window corners."""
    r0, c0 = scr_origin
    out = np.array(screen[r0:r0 + pupil_n, c0:c0 + pupil_n], dtype=np.float64)
    for s, (r, c) in zip(surfaces, origins):
        out -= s[r:r + pupil_n, c:c + pupil_n]
    return out
