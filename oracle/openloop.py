"""Oracle open-loop wavefronts of finite-altitude sources and the LGS uplink tilt (FP64).

Test infrastructure (see the package docstring).

Sec. 4, open-loop generation: the phase screens are piled up, shifted for the
direction of each source; an LGS wavefront is built from 1 to 5 projections of
the beam on sodium sub-layers, each computed with the pupil projection of its
own altitude (the cone effect), and the projection of the beam on the sodium
layer is shifted by the tip-tilt integrated over the upward path.  Reading
O15: a layer at altitude h seen from pupil point r toward direction theta of a
source at altitude H is sampled at p = (1 - h/H) r + h theta (p = r + h theta
for a source at infinity), with bilinear interpolation between screen samples;
the uplink tilt of an LGS is the least-squares tilt of the piled OPD over the
launch beam (diameter d, centred at launcher (1 - h/H) + h theta at altitude
h), and it enters the sensor's wavefront as tilt . r (a spot displacement of
that angle in every sub-aperture).
"""
from __future__ import annotations

import numpy as np


def bilinear(screen, X, Y):
    """Screen value at coordinates (X, Y) in samples (sample (r, c) sits at (c, r)): the usual
    weighted mean of the four surrounding samples."""
    S = np.asarray(screen, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    rows, cols = S.shape
    assert np.all(X >= 0) and np.all(Y >= 0) and np.all(X <= cols - 1) and np.all(Y <= rows - 1)
    ix = np.minimum(np.floor(X).astype(np.int64), cols - 2)
    iy = np.minimum(np.floor(Y).astype(np.int64), rows - 2)
    fx = X - ix
    fy = Y - iy
    return ((1 - fy) * ((1 - fx) * S[iy, ix] + fx * S[iy, ix + 1])
            + fy * ((1 - fx) * S[iy + 1, ix] + fx * S[iy + 1, ix + 1]))


def pupil_coords(pupil_n, dx):
    """Centres of the pupil pixels in metres from the axis: (x[i, j], y[i, j])."""
    c = (np.arange(pupil_n, dtype=np.float64) + 0.5 - pupil_n / 2.0) * dx
    return np.meshgrid(c, c)


def layer_sample(layer, px, py):
    """layer = (screen, spacing_m, altitude_m, x0, y0); (px, py) metres on the layer from the axis."""
    screen, spacing, _, x0, y0 = layer
    return bilinear(screen, x0 + np.asarray(px) / spacing, y0 + np.asarray(py) / spacing)


def project(layers, pupil_n, dx, theta, altitude, tilt=None):
    """Piled OPD of a source in direction theta (radians) at altitude (metres, 0 = infinity)."""
    x, y = pupil_coords(pupil_n, dx)
    opd = np.zeros_like(x)
    for layer in layers:
        h = layer[2]
        s = 1.0 - h / altitude if altitude > 0 else 1.0
        opd += layer_sample(layer, s * x + h * theta[0], s * y + h * theta[1])
    if tilt is not None:
        opd += tilt[0] * x + tilt[1] * y
    return opd


def uplink_samples(d, n_s):
    """Sample offsets (sx, sy) of the launch beam: the n_s x n_s grid over the square of side d,
    points inside the disc of diameter d."""
    c = (np.arange(n_s, dtype=np.float64) + 0.5 - n_s / 2.0) * (d / n_s)
    sx, sy = np.meshgrid(c, c)
    keep = sx ** 2 + sy ** 2 <= 0.25 * d * d
    return sx[keep], sy[keep]


def uplink_tilt(layers, launcher, theta, na_altitude, d, n_s):
    """Least-squares tilt (radians) of the piled OPD over the launch beam: fit a + tx sx + ty sy."""
    sx, sy = uplink_samples(d, n_s)
    opd = np.zeros_like(sx)
    for layer in layers:
        h = layer[2]
        f = h / na_altitude
        cx = launcher[0] * (1 - f) + h * theta[0]
        cy = launcher[1] * (1 - f) + h * theta[1]
        opd += layer_sample(layer, cx + sx, cy + sy)
    A = np.stack([np.ones_like(sx), sx, sy], axis=1)
    coef, *_ = np.linalg.lstsq(A, opd, rcond=None)
    return coef[1], coef[2]
