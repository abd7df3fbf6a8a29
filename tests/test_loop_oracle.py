"""Pins of the oracle's closed loop (CPU): reconstruction of known commands and loop convergence."""
import numpy as np

from gen import configs as G
from oracle import calib as OC
from oracle import dm as OD
from oracle import loop as OL
from oracle import wfs as OW


def test_pinv_reconstructs_known_commands():
    rng = np.random.default_rng(4)
    im = rng.normal(size=(120, 30))
    c = rng.normal(size=30)
    cm = np.linalg.pinv(im)
    got, delta = OL.recon_step(cm, im @ c, 1.0, np.zeros(30))
    assert np.abs(got - c).max() < 1e-10 and np.abs(delta - c).max() < 1e-10


def test_integrator_accumulates():
    rng = np.random.default_rng(5)
    cm = rng.normal(size=(7, 11))
    s = rng.normal(size=11)
    c = np.zeros(7)
    for _ in range(5):
        c, _ = OL.recon_step(cm, s, 0.3, c)
    assert np.abs(c - 5 * 0.3 * cm @ s).max() < 1e-12


def test_loop_converges_on_a_dm_shaped_wavefront():
    """Open-loop wavefront = the DM surface of known commands; push-pull IM of the oracle sensor, CM = pinv.
    With gain 0.5 the commands approach the known ones geometrically: the sign chain of calibration,
    residual (wavefront minus DM) and integrator is right only if the error shrinks."""
    cfg = G.CFG1.replace(pupil_n=80, n_subap=8, flags=0, photons_per_subap=0.0)
    launch = [G.launch_positions(G.CFG1.replace(pupil_n=80, n_subap=8), 1)[0]]
    sensor = OW.Sensor(cfg, 1, launch)
    act = OD.actuators(80, cfg.pupil_dx_m, 0.0, 10, 0.0)
    size = OD.surface_size(80, cfg.pupil_dx_m, 0.0, 0.0)
    im = OC.interaction_matrix(sensor, size, act, range(len(act)), 50e-9, 10, 0.3, 64, 0, 0)
    u, sv, vt = np.linalg.svd(im, full_matrices=False)
    keep = sv > 0.05 * sv[0]
    cm = (vt[keep].T / sv[keep]) @ u[:, keep].T
    rng = np.random.default_rng(6)
    c_true = vt[keep].T @ (vt[keep] @ rng.normal(0, 20e-9, len(act)))   # within the controlled space
    screen = OD.dm_surface(size, act, c_true, 10, 0.3, 64)
    spec = [dict(size=size, alt=0.0, act_xy=act, pitch=10, coupling=0.3, patch=64)]
    hist, _ = OL.closed_loop(sensor, spec, [(0.0, 0.0)], screen, [[(0, 0)]] * 8, cm, 0.5)
    err = [np.linalg.norm(h - c_true) / np.linalg.norm(c_true) for h in hist]
    assert err[0] < 0.6 and err[-1] < 0.02, err
    assert all(b < a for a, b in zip(err, err[1:]))
