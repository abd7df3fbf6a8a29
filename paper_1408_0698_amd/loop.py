"""Closed-loop step on the device (Sec. 3, closed-loop block).

One step: DM surfaces from the current commands, residual wavefront of every
sensor (screen window minus the DM footprints of its direction), slopes of
every sensor, then control-matrix product and pure integrator.  Every step
is a library call on one stream; torch only holds the device buffers.
"""
from __future__ import annotations

import math

from . import shwfs

ARCSEC = math.pi / (180.0 * 3600.0)


class ClosedLoop:
    """plan: WfsPlan of n_wfs sensors; dms: list of (DmPlan, altitude m); directions: per sensor (tx, ty) arcsec;
    screen: float32 device [R][C]; cm: float32 device [n_modes][ld] with n_modes = sum of actuator counts."""

    def __init__(self, plan, dms, directions, screen, cm, gain, seed=0):
        import torch
        self.plan, self.dms, self.dirs = plan, dms, list(directions)
        self.screen, self.cm, self.gain, self.seed = screen, cm, float(gain), seed
        self.n = plan.cfg.pupil_n
        self.n_modes = sum(d.n_act for d, _ in dms)
        if cm.shape[0] != self.n_modes:
            raise ValueError(f"control matrix has {cm.shape[0]} rows, the DMs {self.n_modes} actuators")
        self.n_slopes = plan.n_wfs * 2 * plan.n_valid
        self.coefs = torch.zeros(self.n_modes, device="cuda")
        self.surfs = [torch.zeros((d.size, d.size), device="cuda") for d, _ in dms]
        self.res = torch.empty((plan.n_wfs, self.n, self.n), device="cuda")
        self.slopes = torch.empty((1, plan.n_wfs, 2, plan.n_valid), device="cuda")
        self.recon = shwfs.ReconPlan(self.n_modes, self.n_slopes)
        dx = plan.cfg.pupil_dx_m
        self.dm_o = []
        for (tx, ty) in self.dirs:
            row = []
            for d, alt in dms:
                sy = int(math.floor(alt * ty * ARCSEC / dx + 0.5))
                sx = int(math.floor(alt * tx * ARCSEC / dx + 0.5))
                row.append((d.size // 2 - self.n // 2 + sy, d.size // 2 - self.n // 2 + sx))
            self.dm_o.append(row)

    def step(self, scr_origins, frame, stream=None):
        """One loop step; scr_origins[w] = (row, col) of sensor w's screen window.  Returns the slopes."""
        off = 0
        for (d, _), sf in zip(self.dms, self.surfs):
            d.surface(self.coefs[off:off + d.n_act], sf, stream=stream)
            off += d.n_act
        shwfs.residual_opd(self.screen, self.surfs, self.n, scr_origins, self.dm_o, self.res, stream=stream)
        self.plan.measure(self.res.unsqueeze(0), self.slopes, seed=self.seed, frame0=frame, stream=stream)
        self.recon.step(self.cm, self.slopes.view(-1), self.gain, self.coefs, stream=stream)
        return self.slopes
