"""GPU parity of the large-sub-aperture path (FFT 512: 2x2 sub-apertures of 400x400 px)."""
import numpy as np
import pytest

from gen import configs as G
from gen import screens as S
from oracle import wfs as OW
from tests.test_gpu_wfs import assert_images_close, assert_slopes_close, check_noisy, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _opd(nf, nw, scale=1.0):
    return (S.lgs39m_opd(nf, nw, pupil_n=800) * scale).astype(np.float32)


def test_ngs512_noise_free_parity(torch_dev):
    cfg = G.CFG4_NGS.replace(flags=0)
    opd = _opd(1, 3, 0.05)
    got = run_gpu(torch_dev, cfg, 3, None, opd)
    want = OW.Sensor(cfg, 3).measure(opd)
    assert_images_close(got["images"], want["images"])
    assert_slopes_close(got["slopes"], want["slopes"])


def test_ngs512_noisy_parity(torch_dev):
    cfg = G.CFG4_NGS
    opd = _opd(1, 3, 0.05)
    seed = 4242
    got = run_gpu(torch_dev, cfg, 3, None, opd, seed=seed, frame0=3)
    sens = OW.Sensor(cfg, 3)
    want = sens.measure(opd, seed=seed, frame0=3)
    check_noisy(cfg, 3, None, got, want, seed, 3, lambda w: w * sens.n_valid + np.arange(sens.n_valid))


def test_ngs512_unpadded_size_and_flat(torch_dev):
    """A sub-aperture size that does not divide 512 (pupil 200, 100 px), flat and tilted."""
    cfg = G.CFG4_NGS.replace(pupil_n=200, flags=0, photons_per_subap=0.0, obstruction=0.0)
    flat = np.zeros((1, 1, 200, 200), np.float32)
    got = run_gpu(torch_dev, cfg, 1, None, flat)
    assert np.abs(got["slopes"]).max() < 1e-4
    opd = _opd(1, 1)[:, :, :200, :200] * 0.02
    got = run_gpu(torch_dev, cfg, 1, None, opd)
    want = OW.Sensor(cfg, 1).measure(opd)
    assert_images_close(got["images"], want["images"])
    assert_slopes_close(got["slopes"], want["slopes"])


def test_ngs512_chunking_is_invisible(torch_dev):
    """More work items than one workspace chunk: every frame equals that frame run alone."""
    cfg = G.CFG4_NGS
    nf = 8
    opd = _opd(nf, 3, 0.05)
    many = run_gpu(torch_dev, cfg, 3, None, opd, seed=9, frame0=100)
    for f in (0, 5, 7):
        one = run_gpu(torch_dev, cfg, 3, None, opd[f:f + 1], seed=9, frame0=100 + f)
        assert np.array_equal(many["slopes"][f], one["slopes"][0])
        assert np.array_equal(many["images"][f], one["images"][0])
