"""Push-pull interaction-matrix calibration (Sec. 3 interaction-matrix block; Sec. 5).

Each mode (the influence function of one DM actuator) is pushed and pulled
by +/- amplitude on the pupil, every sensor of the plan measures both
frames, and the interaction-matrix column is (s+ - s-) / (2 amplitude).
All steps are library kernels: influence-function OPD frames, the fused
measurement (one launch per chunk of modes, every sensor of the plan
seeing the same pupil OPD through a zero sensor stride), and the
push-pull combination into the matrix.
"""
from __future__ import annotations

import numpy as np

from . import shwfs


def interaction_matrix(plan: "shwfs.WfsPlan", dm: "shwfs.DmPlan", acts, amplitude_m: float, row0: int, col0: int,
                       chunk: int = 512, stream=None):
    """Interaction matrix [n_wfs * 2 * n_valid][len(acts)] (detector pixels per metre of OPD), device FP32."""
    import torch
    n_modes = len(acts)
    N = plan.cfg.pupil_n
    n_slopes = plan.n_wfs * 2 * plan.n_valid
    im = torch.empty((n_slopes, n_modes), device="cuda")
    acts = np.asarray(acts, dtype=np.int32)
    for m0 in range(0, n_modes, chunk):
        n = min(chunk, n_modes - m0)
        act = torch.from_numpy(np.repeat(acts[m0:m0 + n], 2)).cuda()
        amp = torch.from_numpy(np.tile(np.array([amplitude_m, -amplitude_m], np.float32), n)).cuda()
        opd = torch.empty((2 * n, N, N), device="cuda")
        dm.influence_opd(act, amp, row0, col0, N, opd, stream=stream)
        slopes = torch.empty((2 * n, plan.n_wfs, 2, plan.n_valid), device="cuda")
        plan.measure(opd.unsqueeze(1).expand(-1, plan.n_wfs, -1, -1), slopes, stream=stream)
        shwfs.push_pull(slopes.view(2 * n, n_slopes), n, 1.0 / (2.0 * amplitude_m), im[:, m0:], stream=stream)
    return im
