"""GPU parity of the open-loop geometry (cone-effect projection, uplink tilt) and of the PSF
extras (encircled energy, resampling, colour-weighted PSF) against the FP64 oracle, through the
C ABI.

Bars: projected OPD within 1e-6 of the largest |OPD| (FP32 output of FP64 sums); uplink tilt
within 1e-9 relative (FP64 on both sides); encircled energy within 1e-9 (FP64 sums of the same
FP32 values); resampled and colour-weighted PSFs within 1e-5 of their maximum.  Inputs are
seeded on the host; no expected value comes from the GPU.
"""
import numpy as np
import pytest

from gen import configs as G
from gen import screens as S
from oracle import openloop as OL
from oracle import psf as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _screens(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r, c in shapes:
        # smooth random OPD (metres): a few sinusoids plus white noise, so interpolation matters
        Y, X = np.mgrid[0:r, 0:c].astype(np.float64)
        f = sum(rng.normal() * np.sin(rng.uniform(0.01, 0.3) * X + rng.uniform(0.01, 0.3) * Y + rng.uniform(0, 6.3))
                for _ in range(6))
        out.append((1e-7 * f + 2e-8 * rng.normal(size=(r, c))).astype(np.float32))
    return out


def _layers(torch, screens, params):
    dev = [torch.from_numpy(s).cuda() for s in screens]
    gpu = [(d, *p) for d, p in zip(dev, params)]
    host = [(s.astype(np.float64), *p) for s, p in zip(screens, params)]
    return gpu, host


PARAMS = [(0.1, 0.0, 150.3, 149.8), (0.15, 4000.0, 150.0, 150.0), (0.2, 12700.0, 149.6, 150.2)]


@pytest.mark.parametrize("with_tilt", [False, True])
def test_projection_parity(torch_dev, with_tilt):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("projection parity, tilt", with_tilt, flush=True)
    scr = _screens([(300, 300), (300, 310), (320, 300)], 11)
    gpu, host = _layers(torch, scr, PARAMS)
    N, dx = 96, 0.1
    targets = [(2e-4, -1e-4, 0.0), (2e-4, 0.0, 88500.0), (2e-4, 0.0, 90000.0), (-1e-4, 3e-4, 91500.0),
               (0.0, 0.0, 0.0)]
    tilt = np.array([[1e-7, -2e-7], [0, 0], [3e-7, 1e-7], [-1e-7, 0.0], [0.0, 5e-8]])
    d_tilt = torch.from_numpy(tilt).cuda() if with_tilt else None
    out = torch.full((len(targets), N, N), float("nan"), device="cuda")
    shwfs.project_layers(gpu, N, dx, targets, out, tilt=d_tilt)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    for t, (tx, ty, H) in enumerate(targets):
        want = OL.project(host, N, dx, (tx, ty), H, tilt[t] if with_tilt else None)
        assert np.abs(got[t] - want).max() <= 1e-6 * np.abs(want).max(), t


def test_projection_full_size_sampled(torch_dev):
    """The open-loop shape of a frame: 6 LGS x 3 sodium sub-layers (18 targets) from three 2048^2
    layers onto the 800^2 pupil; the oracle checks three targets in full."""
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("projection full size", flush=True)
    cfg = G.CFG1
    scr = [S.screen_opd_m(2048, cfg.pupil_dx_m, G.SCREEN_SEED + k).astype(np.float32) for k in range(3)]
    params = [(cfg.pupil_dx_m, h, 1023.5, 1023.5) for h in (0.0, 4000.0, 12700.0)]
    gpu, host = _layers(torch, scr, params)
    lgs_dir = [(45.0 * G.ARCSEC * np.cos(a), 45.0 * G.ARCSEC * np.sin(a)) for a in np.arange(6) * np.pi / 3]
    alts = [cfg.na_height_m + dh for dh in G.SODIUM[0]]
    targets = [(tx, ty, H) for tx, ty in lgs_dir for H in alts]
    out = torch.empty((18, cfg.pupil_n, cfg.pupil_n), device="cuda")
    shwfs.project_layers(gpu, cfg.pupil_n, cfg.pupil_dx_m, targets, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for t in (0, 7, 17):
        want = OL.project(host, cfg.pupil_n, cfg.pupil_dx_m, targets[t][:2], targets[t][2])
        assert np.abs(got[t] - want).max() <= 1e-6 * np.abs(want).max(), t


def test_uplink_tilt_parity(torch_dev):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("uplink tilt parity", flush=True)
    cfg = G.CFG1
    scr = [S.screen_opd_m(2048, cfg.pupil_dx_m, G.SCREEN_SEED + 10 + k).astype(np.float32) for k in range(3)]
    params = [(cfg.pupil_dx_m, h, 1023.5, 1023.5) for h in (0.0, 4000.0, 12700.0)]
    gpu, host = _layers(torch, scr, params)
    launch = G.launch_positions(cfg, 6)
    lgs = [(lx, ly, 45.0 * G.ARCSEC * np.cos(a), 45.0 * G.ARCSEC * np.sin(a), cfg.na_height_m)
           for (lx, ly), a in zip(launch, np.arange(6) * np.pi / 3)]
    out = torch.zeros((6, 2), dtype=torch.float64, device="cuda")
    shwfs.uplink_tilt(gpu, lgs, 0.4, 48, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for k, g in enumerate(lgs):
        want = np.array(OL.uplink_tilt(host, g[:2], g[2:4], g[4], 0.4, 48))
        assert np.abs(got[k] - want).max() <= 1e-9 * np.abs(want).max() + 1e-20, k
    assert np.all(np.abs(got) > 0)


def _psf_like(M, seed):
    """A seeded positive PSF-shaped array: an Airy core, a halo and noise (host)."""
    rng = np.random.default_rng(seed)
    d = np.arange(M, dtype=np.float64) - M // 2
    r = np.hypot(d[None, :], d[:, None]) * 0.2 + 1e-9
    from scipy.special import j1
    airy = (2 * j1(r) / r) ** 2
    halo = 1e-3 / (1 + (r / 30.0) ** 2)
    return (0.3 * airy + halo + 1e-5 * rng.random((M, M))).astype(np.float32)


def test_encircled_energy_parity(torch_dev):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("encircled energy parity", flush=True)
    cfg = G.CFG3
    plan = shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, cfg.fft_m, cfg.wavelength_m)
    P = np.stack([_psf_like(cfg.fft_m, 3), _psf_like(cfg.fft_m, 4)[::-1].copy()])
    radii = [0.0, 0.5, 1.0, 2.5, 7.0, 19.9, 20.0, 64.0, 300.0, 799.0, 1200.0, 5000.0]
    ee = plan.encircled_energy(torch.from_numpy(P).cuda(), radii)
    torch.cuda.synchronize()
    got = ee.cpu().numpy()
    for s in range(2):
        want = OP.encircled_energy(P[s].astype(np.float64), radii)
        assert np.abs(got[s] - want).max() < 1e-9, s
    assert got[0, -1] == 1.0
    # the same call twice gives the same bits (fixed summation order)
    again = plan.encircled_energy(torch.from_numpy(P).cuda(), radii).cpu().numpy()
    assert np.array_equal(again, got)


@pytest.mark.parametrize("scale", [0.8, 1.0, 1.3])
def test_resample_parity(torch_dev, scale):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("resample parity", scale, flush=True)
    M = 256
    P = _psf_like(M, 9)
    base = np.random.default_rng(1).random((M, M)).astype(np.float32)
    dst = torch.from_numpy(base.copy()).cuda()
    shwfs.psf_resample_accumulate(torch.from_numpy(P).cuda(), scale, 0.7, dst)
    torch.cuda.synchronize()
    want = base.astype(np.float64) + 0.7 * OP.resample(P.astype(np.float64), scale)
    assert np.abs(dst.cpu().numpy() - want).max() <= 1e-5 * np.abs(want).max()


def test_polychromatic_psf_parity(torch_dev):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("polychromatic parity", flush=True)
    lams, w = (1.65e-6, 1.5e-6, 1.8e-6), (0.5, 0.2, 0.3)
    cfgs = [G.PsfConfig(pupil_n=64, pupil_dx_m=39.0 / 64, wavelength_m=l) for l in lams]
    scr = S.screen_opd_m(2048, 4.875e-2, G.SCREEN_SEED)
    opd = np.stack([scr[:64, t:t + 64] * 0.3 for t in (0, 5)]).astype(np.float32)
    plans = [shwfs.PsfPlan(c.pupil_n, c.pupil_dx_m, c.obstruction, c.fft_m, c.wavelength_m) for c in cfgs]
    out = torch.zeros((1600, 1600), device="cuda")
    sr = torch.zeros((3, 2), device="cuda")
    shwfs.polychromatic_psf(plans, w, torch.from_numpy(opd).cuda(), out, strehl=sr)
    torch.cuda.synchronize()
    want = OP.polychromatic(cfgs, w, opd.astype(np.float64))
    got = out.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-5 * want.max()
    # the on-axis value of the colour-weighted PSF is the weighted sum of the per-wavelength Strehl ratios
    assert abs(got[800, 800] - float((torch.tensor(w, device="cuda")[:, None] * sr).sum())) < 1e-5 * got[800, 800]


def test_lgs_frame_from_layers_parity(torch_dev):
    """End to end: uplink tilts, cone-effect wavefronts of every sodium sub-layer, sodium measurement,
    against the oracle's projection and sensor (noise off)."""
    from oracle import wfs as OW
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("LGS frame from layers", flush=True)
    cfg = G.CFG1.replace(pupil_n=130, n_subap=13, flags=0)
    n_wfs = 6
    launch = G.launch_positions(cfg, n_wfs)
    scr = [(S.screen_opd_m(512, cfg.pupil_dx_m, G.SCREEN_SEED + 20 + k)[:400, :400] * 0.5).astype(np.float32)
           for k in range(3)]
    params = [(cfg.pupil_dx_m, h, 199.5, 200.5) for h in (0.0, 4000.0, 12700.0)]
    gpu, host = _layers(torch, scr, params)
    dirs = [(45.0 * G.ARCSEC * np.cos(a), 45.0 * G.ARCSEC * np.sin(a)) for a in np.arange(n_wfs) * np.pi / 3]
    lgs = [(lx, ly, tx, ty, cfg.na_height_m) for (lx, ly), (tx, ty) in zip(launch, dirs)]
    dh = G.SODIUM[0]
    targets = [(tx, ty, cfg.na_height_m + d) for tx, ty in dirs for d in dh]
    tilt = torch.zeros((n_wfs, 2), dtype=torch.float64, device="cuda")
    shwfs.uplink_tilt(gpu, lgs, 0.4, 32, tilt)
    tilt_t = tilt.repeat_interleave(len(dh), dim=0).contiguous()
    opd = torch.empty((1, n_wfs, len(dh), cfg.pupil_n, cfg.pupil_n), device="cuda")
    shwfs.project_layers(gpu, cfg.pupil_n, cfg.pupil_dx_m, targets, opd.view(-1, cfg.pupil_n, cfg.pupil_n),
                         tilt=tilt_t)
    plan = shwfs.WfsPlan(cfg, n_wfs, launch, sodium=G.SODIUM)
    sl = torch.full((1, n_wfs, 2, plan.n_valid), float("nan"), device="cuda")
    im = torch.full((1, n_wfs, plan.n_valid, 16, 16), float("nan"), device="cuda")
    plan.measure_sodium(opd, sl, im)
    torch.cuda.synchronize()
    # oracle: tilts, wavefronts and sensor from the same host layers
    want_opd = np.empty((1, n_wfs, len(dh), cfg.pupil_n, cfg.pupil_n))
    for w, g in enumerate(lgs):
        t = OL.uplink_tilt(host, g[:2], g[2:4], g[4], 0.4, 32)
        for j, d in enumerate(dh):
            want_opd[0, w, j] = OL.project(host, cfg.pupil_n, cfg.pupil_dx_m, g[2:4], cfg.na_height_m + d, t)
    want = OW.Sensor(cfg, n_wfs, launch, sodium=G.SODIUM).measure(want_opd)
    from test_gpu_wfs import assert_images_close, assert_slopes_close
    assert_images_close(im.cpu().numpy().astype(np.float64), want["images"])
    assert_slopes_close(sl.cpu().numpy().astype(np.float64), want["slopes"])


def test_geometry_edge_cases(torch_dev):
    """No targets is a no-op; bad arguments raise before any launch; a single-wavelength
    colour-weighted PSF is the plain accumulation; a single 2-D PSF and a zero radius."""
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    print("geometry edge cases", flush=True)
    scr = _screens([(64, 64)], 5)
    gpu, _ = _layers(torch, scr, [(0.1, 0.0, 32.0, 32.0)])
    out = torch.full((1, 16, 16), 7.0, device="cuda")
    shwfs.project_layers(gpu, 16, 0.1, [], out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    with pytest.raises(shwfs.ShwError):
        shwfs.project_layers(gpu, 16, 0.1, [(0.0, 0.0, -1.0)], out)   # negative altitude
    with pytest.raises(shwfs.ShwError):
        shwfs.project_layers(gpu, 200, 0.1, [(0.0, 0.0, 0.0)], torch.empty((1, 200, 200), device="cuda"))
    with pytest.raises(shwfs.ShwError):
        shwfs.uplink_tilt(gpu, [(0.0, 0.0, 0.0, 0.0, 90000.0)], 0.4, 1, torch.empty((1, 2), dtype=torch.float64,
                                                                                    device="cuda"))
    cfg = G.PsfConfig(pupil_n=64, pupil_dx_m=39.0 / 64)
    plan = shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, cfg.fft_m, cfg.wavelength_m)
    opd = torch.from_numpy((S.screen_opd_m(512, 0.1)[:64, :64] * 0.2).astype(np.float32)[None]).cuda()
    a = torch.zeros((1600, 1600), device="cuda")
    plan.accumulate(opd, a)
    b = torch.zeros((1600, 1600), device="cuda")
    shwfs.polychromatic_psf([plan], [1.0], opd, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ee = plan.encircled_energy(a, [0.0])
    torch.cuda.synchronize()
    assert ee.shape == (1,)
    assert abs(float(ee[0]) - float(a[800, 800]) / float(a.double().sum())) < 1e-9
    with pytest.raises(shwfs.ShwError):
        shwfs.psf_resample_accumulate(a, 1.0, 1.0, a)   # source and destination overlap
