"""Oracle closed-loop step (FP64).

Test infrastructure (see the package docstring).

Sec. 3, closed-loop block: the residual wavefront (open-loop wavefront minus
the DMs) is measured by the sensors, the slope vectors are multiplied by the
control matrix, giving modal increments, and a pure integrator accumulates
them into the commands.  Reading O14: the modes are the actuators'
influence functions (the modal base of the paper is out of scope), the
increment is added (the residual is wavefront minus DM and the interaction
matrix registers slopes per positive command), and the gain multiplies it.
"""
from __future__ import annotations

import numpy as np

from . import dm as D


def recon_step(cm, slopes, gain, coefs):
    """delta = CM s; coefs + gain delta.  Returns (new coefs, delta)."""
    delta = np.asarray(cm, dtype=np.float64) @ np.asarray(slopes, dtype=np.float64)
    return np.asarray(coefs, dtype=np.float64) + gain * delta, delta


def dm_origins(pupil_n, dx_m, dms, direction_arcsec):
    """(row, col) window corners of the pupil footprint of one direction on each DM (reading O12)."""
    tx, ty = direction_arcsec
    out = []
    for size, alt in dms:
        out.append((size // 2 - pupil_n // 2 + D.footprint_shift_px(alt, ty, dx_m),
                    size // 2 - pupil_n // 2 + D.footprint_shift_px(alt, tx, dx_m)))
    return out


def closed_loop(sensor, dm_specs, directions, screen, scr_origins, cm, gain, seed=0, coefs0=None):
    """Run len(scr_origins) loop steps.

    dm_specs: list of dict(size, alt, act_xy, pitch, coupling, patch); directions: per sensor (tx, ty)
    arcsec; scr_origins[t][w]: screen window corner of sensor w at step t.  Returns (coefs after
    every step [T][n_modes], slopes of every step [T][n_slopes]).
    """
    cfg = sensor.cfg
    n = cfg.pupil_n
    n_modes = sum(len(d["act_xy"]) for d in dm_specs)
    coefs = np.zeros(n_modes) if coefs0 is None else np.array(coefs0, dtype=np.float64)
    hist_c, hist_s = [], []
    for t, origins in enumerate(scr_origins):
        surfs, off = [], 0
        for d in dm_specs:
            k = len(d["act_xy"])
            surfs.append(D.dm_surface(d["size"], d["act_xy"], coefs[off:off + k], d["pitch"], d["coupling"],
                                      d["patch"]))
            off += k
        opd = np.stack([D.residual_opd(screen, origins[w], surfs,
                                       dm_origins(n, cfg.pupil_dx_m, [(d["size"], d["alt"]) for d in dm_specs],
                                                  directions[w]), n)
                        for w in range(sensor.n_wfs)])
        s = sensor.measure(opd[None], seed=seed, frame0=t)["slopes"][0].ravel()
        coefs, _ = recon_step(cm, s, gain, coefs)
        hist_c.append(coefs.copy())
        hist_s.append(s)
    return np.array(hist_c), np.array(hist_s)
