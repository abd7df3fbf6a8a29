"""Sodium sub-layer form of the LGS sensor on the GPU against the FP64 oracle (through the C ABI).

Bars as for the single-kernel form: images within 1e-4 of the sub-aperture
maximum, slopes within 1e-3 detector pixel; noisy counts equal except at
explained ties.
"""
import numpy as np
import pytest

from gen import configs as G
from gen import screens as S
from oracle import wfs as OW
from test_gpu_wfs import assert_images_close, assert_slopes_close, check_noisy, small_lgs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_sodium(torch, cfg, n_wfs, launch, sodium, opd, seed=0, frame0=0, per_layer=False):
    from paper_1408_0698_amd import shwfs
    plan = shwfs.WfsPlan(cfg, n_wfs, launch, sodium=sodium)
    d = torch.from_numpy(np.ascontiguousarray(opd, dtype=np.float32)).cuda()
    nf = opd.shape[0]
    if not per_layer:
        d = d.unsqueeze(2).expand(-1, -1, len(sodium[0]), -1, -1)
    sl = torch.full((nf, n_wfs, 2, plan.n_valid), float("nan"), device="cuda")
    im = torch.full((nf, n_wfs, plan.n_valid, cfg.det_n, cfg.det_n), float("nan"), device="cuda")
    plan.measure_sodium(d, sl, im, seed=seed, frame0=frame0)
    torch.cuda.synchronize()
    return dict(slopes=sl.cpu().numpy().astype(np.float64), images=im.cpu().numpy().astype(np.float64), plan=plan)


@pytest.mark.parametrize("ns,n_wfs", [(13, 6), (17, 2)])
def test_shared_wavefront_parity(torch_dev, ns, n_wfs):
    cfg = small_lgs(ns, flags=0)
    launch = G.launch_positions(cfg, n_wfs)
    opd = S.lgs39m_opd(2, n_wfs, pupil_n=cfg.pupil_n)
    got = run_sodium(torch_dev, cfg, n_wfs, launch, G.SODIUM, opd)
    want = OW.Sensor(cfg, n_wfs, launch, sodium=G.SODIUM).measure(opd)
    assert_images_close(got["images"], want["images"])
    assert_slopes_close(got["slopes"], want["slopes"])


def test_one_wavefront_per_sublayer_parity(torch_dev):
    """Five sub-layers, each with its own wavefront (sub-layer stride of one pupil)."""
    cfg = small_lgs(12, flags=0)
    launch = G.launch_positions(cfg, 3)
    sod = G.sodium_profile(5, G.SODIUM_THICKNESS_M)
    opd = np.stack([S.lgs39m_opd(1, 3, frame0=7 * j, pupil_n=cfg.pupil_n) for j in range(5)], axis=2)
    got = run_sodium(torch_dev, cfg, 3, launch, sod, opd, per_layer=True)
    want = OW.Sensor(cfg, 3, launch, sodium=sod).measure(opd)
    assert_images_close(got["images"], want["images"])
    assert_slopes_close(got["slopes"], want["slopes"])


def test_noisy_parity(torch_dev):
    cfg = small_lgs(13)
    launch = G.launch_positions(cfg, 6)
    opd = S.lgs39m_opd(1, 6, pupil_n=cfg.pupil_n)
    seed = G.NOISE_SEED + 77
    got = run_sodium(torch_dev, cfg, 6, launch, G.SODIUM, opd, seed=seed, frame0=3)
    sens = OW.Sensor(cfg, 6, launch, sodium=G.SODIUM)
    want = sens.measure(opd, seed=seed, frame0=3)
    check_noisy(cfg, 6, launch, got, want, seed, 3, lambda w: w * sens.n_valid + np.arange(sens.n_valid))


def test_single_layer_at_focus_equals_round_kernel_plan(torch_dev):
    """One sub-layer at the focus height is the single-kernel form with no elongation: bitwise equal."""
    from paper_1408_0698_amd import shwfs
    cfg = small_lgs(13)
    launch = G.launch_positions(cfg, 6)
    opd = S.lgs39m_opd(1, 6, pupil_n=cfg.pupil_n)
    a = run_sodium(torch_dev, cfg, 6, launch, ([0.0], [1.0]), opd, seed=9)
    plan = shwfs.WfsPlan(cfg.replace(elong_max_arcsec=1e-12), 6, launch)
    d = torch_dev.from_numpy(opd).cuda()
    sl = torch_dev.zeros((1, 6, 2, plan.n_valid), device="cuda")
    im = torch_dev.zeros((1, 6, plan.n_valid, 16, 16), device="cuda")
    plan.measure(d, sl, im, seed=9)
    torch_dev.cuda.synchronize()
    assert np.array_equal(a["images"], im.cpu().numpy().astype(np.float64))
    assert np.array_equal(a["slopes"], sl.cpu().numpy().astype(np.float64))


def test_plain_measure_on_sodium_plan_shares_the_wavefront(torch_dev):
    cfg = small_lgs(12, flags=0)
    launch = G.launch_positions(cfg, 2)
    opd = S.lgs39m_opd(1, 2, pupil_n=cfg.pupil_n)
    a = run_sodium(torch_dev, cfg, 2, launch, G.SODIUM, opd)
    d = torch_dev.from_numpy(opd).cuda()
    sl = torch_dev.zeros((1, 2, 2, a["plan"].n_valid), device="cuda")
    a["plan"].measure(d, sl)
    torch_dev.cuda.synchronize()
    assert np.array_equal(a["slopes"], sl.cpu().numpy().astype(np.float64))


def test_variants_agree(torch_dev):
    """Within a row-transform family the variants agree (split rows: 1, 2; band-limited: 3, 4): images
    bitwise, slopes bitwise when the centroid is taken in the same kernel (variant 1 sums in FP64 in
    the fused kernel, 2-4 in FP32 in the detector kernel: within 1e-4 px); across families the
    noise-free images agree to FP32 rounding."""
    from paper_1408_0698_amd import shwfs
    cfg = small_lgs(13)
    launch = G.launch_positions(cfg, 6)
    opd = S.lgs39m_opd(1, 6, pupil_n=cfg.pupil_n)
    d = torch_dev.from_numpy(opd).cuda().unsqueeze(2).expand(-1, -1, 3, -1, -1)
    outs = {}
    for c in (cfg, cfg.replace(flags=0)):
        plan = shwfs.WfsPlan(c, 6, launch, sodium=G.SODIUM)
        assert plan.n_variants == 5
        for v in range(plan.n_variants):
            plan.set_variant(v)
            sl = torch_dev.zeros((1, 6, 2, plan.n_valid), device="cuda")
            im = torch_dev.zeros((1, 6, plan.n_valid, 16, 16), device="cuda")
            plan.measure_sodium(d, sl, im, seed=4)
            outs[(c.flags, v)] = (sl, im)
    torch_dev.cuda.synchronize()
    for fl in (cfg.flags, 0):
        for x, y in ((1, 2), (3, 4)):
            assert torch_dev.equal(outs[(fl, x)][1], outs[(fl, y)][1]), (fl, x, y)
            if x == 1:
                assert (outs[(fl, x)][0] - outs[(fl, y)][0]).abs().max().item() < 1e-4, (fl, x, y)
            else:
                assert torch_dev.equal(outs[(fl, x)][0], outs[(fl, y)][0]), (fl, x, y)
    a = outs[(0, 0)][1].cpu().numpy()
    for v in (1, 3):
        b = outs[(0, v)][1].cpu().numpy()
        assert (abs(a - b) / abs(a).max(axis=(-1, -2), keepdims=True)).max() < 1e-6, v


@pytest.mark.parametrize("variant", [2, 4])
def test_variant_parity(torch_dev, variant):
    """Split-row and band-limited sodium kernels against the oracle, five sub-layers of their own."""
    cfg = small_lgs(12, flags=0)
    launch = G.launch_positions(cfg, 3)
    sod = G.sodium_profile(5, G.SODIUM_THICKNESS_M)
    opd = np.stack([S.lgs39m_opd(1, 3, frame0=7 * j, pupil_n=cfg.pupil_n) for j in range(5)], axis=2)
    from paper_1408_0698_amd import shwfs
    plan = shwfs.WfsPlan(cfg, 3, launch, sodium=sod)
    plan.set_variant(variant)
    dd = torch_dev.from_numpy(np.ascontiguousarray(opd, dtype=np.float32)).cuda()
    sl = torch_dev.zeros((1, 3, 2, plan.n_valid), device="cuda")
    im = torch_dev.zeros((1, 3, plan.n_valid, 16, 16), device="cuda")
    plan.measure_sodium(dd, sl, im)
    torch_dev.cuda.synchronize()
    want = OW.Sensor(cfg, 3, launch, sodium=sod).measure(opd)
    assert_images_close(im.cpu().numpy().astype(np.float64), want["images"])
    assert_slopes_close(sl.cpu().numpy().astype(np.float64), want["slopes"])


def test_full_frame_sampled(torch_dev):
    """The 6-LGS 80x80 frame with three sub-layers; the oracle recomputes a sample of sub-apertures."""
    cfg = G.CFG1.replace(flags=0)
    launch = G.launch_positions(cfg, 6)
    opd = S.lgs39m_opd(1, 6)
    got = run_sodium(torch_dev, cfg, 6, launch, G.SODIUM, opd)
    sens = OW.Sensor(cfg, 6, launch, sodium=G.SODIUM)
    sub = np.unique(np.concatenate([np.random.default_rng(2).choice(sens.n_valid, 60, replace=False),
                                    [0, sens.n_valid - 1]]))
    want = sens.measure(opd, subset=sub)
    assert_images_close(got["images"][:, :, sub], want["images"])
    assert_slopes_close(got["slopes"][..., sub], want["slopes"])
    flux = got["images"].sum(axis=(-1, -2))
    from oracle import geometry as OG
    _, illum = OG.subap_table(cfg)
    assert np.abs(flux - cfg.photons_per_subap * illum[None, None, :]).max() < 1e-3 * cfg.photons_per_subap
