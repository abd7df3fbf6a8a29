"""Oracle push-pull interaction matrix (FP64).

Test infrastructure (see the package docstring).

Sec. 3 interaction-matrix block: the modes of the base are used to register
the slopes measured by the WFS; Sec. 5: the calibration was a modal
push-pull.  Reading: the modes are the DM's influence functions, pushed and
pulled by +/- a on the pupil window, column = (s+ - s-) / (2 a).
"""
from __future__ import annotations

import numpy as np

from . import dm as D


def influence_window(size, act_xy, k, amp, pitch, coupling, patch, row0, col0, pupil_n):
    surf = D.dm_surface(size, act_xy[k:k + 1], [amp], pitch, coupling, patch)
    return surf[row0:row0 + pupil_n, col0:col0 + pupil_n]


def interaction_matrix(sensor, size, act_xy, acts, amp, pitch, coupling, patch, row0, col0, subset=None):
    """[n_wfs * 2 * S][len(acts)]; every sensor sees the same pupil OPD."""
    cols = []
    n = sensor.cfg.pupil_n
    for k in acts:
        res = []
        for a in (amp, -amp):
            opd = influence_window(size, act_xy, k, a, pitch, coupling, patch, row0, col0, n)
            opd = np.repeat(opd[None, None].astype(np.float32), sensor.n_wfs, axis=1)
            res.append(sensor.measure(opd, subset=subset)["slopes"][0])
        cols.append(((res[0] - res[1]) / (2.0 * amp)).ravel())
    return np.stack(cols, axis=1)
