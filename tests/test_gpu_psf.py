"""GPU parity of psf_accumulate against the FP64 oracle (through the C ABI).

Bar: accumulated PSF within 1e-4 of its maximum, Strehl within 1e-4 of
the oracle's on-axis value; closed forms at full size (Strehl of every
frame against |sum A e^{i phi}|^2 / (sum A)^2, Parseval sum P = M^2 / sum A).
"""
import numpy as np
import pytest

from gen import configs as G
from gen import screens as S
from oracle import geometry as OG
from oracle import psf as OP

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(cfg):
    from paper_1408_0698_amd import shwfs
    return shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, cfg.fft_m, cfg.wavelength_m)


def _opd(n_frames, pupil_n, scale=1.0, seed=S.C.SCREEN_SEED):
    scr = S.screen_opd_m(2048, 4.875e-2, seed)
    return np.stack([scr[:pupil_n, t:t + pupil_n] * scale for t in range(n_frames)]).astype(np.float32)


def run_gpu(torch, cfg, opd, acc0=None):
    plan = _plan(cfg)
    d = torch.from_numpy(opd).cuda()
    acc = torch.zeros((cfg.fft_m, cfg.fft_m), device="cuda") if acc0 is None else acc0.clone()
    sr = torch.full((opd.shape[0],), float("nan"), device="cuda")
    plan.accumulate(d, acc, sr)
    torch.cuda.synchronize()
    return acc.cpu().numpy().astype(np.float64), sr.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("pupil_n,nf,scale", [(100, 3, 0.05), (123, 9, 0.2), (40, 1, 1.0)])
def test_small_pupil_parity(torch_dev, pupil_n, nf, scale):
    cfg = G.PsfConfig(pupil_n=pupil_n, pupil_dx_m=39.0 / pupil_n)
    opd = _opd(nf, pupil_n, scale)
    acc, sr = run_gpu(torch_dev, cfg, opd)
    want_acc, want_sr = OP.psf_accumulate(cfg, opd)
    assert np.abs(acc - want_acc).max() <= TOL * want_acc.max()
    assert np.abs(sr - want_sr).max() <= TOL * max(want_sr.max(), 1e-3)


def test_full_pupil_two_frames_and_closed_forms(torch_dev):
    cfg = G.CFG3
    opd = _opd(2, 800, 0.1)
    acc, sr = run_gpu(torch_dev, cfg, opd)
    want_acc, want_sr = OP.psf_accumulate(cfg, opd)
    assert np.abs(acc - want_acc).max() <= TOL * want_acc.max()
    for f in range(2):
        assert abs(sr[f] - OP.strehl_direct(cfg, opd[f])) <= TOL * max(sr[f], 1e-3)
    nlit = OG.pupil_mask(800, 0.14).sum()
    assert abs(acc.sum() - 2 * cfg.fft_m ** 2 / nlit) < 1e-3 * acc.sum()


def test_full_pupil_strehl_series(torch_dev):
    """20 frames of the science workload: Strehl of each frame equals the transform-free closed form."""
    cfg = G.CFG3
    opd = _opd(20, 800, 0.08)
    acc, sr = run_gpu(torch_dev, cfg, opd)
    want = np.array([OP.strehl_direct(cfg, o) for o in opd])
    assert np.abs(sr - want).max() <= TOL * want.max()
    nlit = OG.pupil_mask(800, 0.14).sum()
    assert abs(acc.sum() - 20 * cfg.fft_m ** 2 / nlit) < 1e-3 * acc.sum()


def test_flat_wavefront_is_diffraction_limited(torch_dev):
    cfg = G.CFG3
    acc, sr = run_gpu(torch_dev, cfg, np.zeros((1, 800, 800), np.float32))
    assert abs(sr[0] - 1.0) < 1e-5
    c = cfg.fft_m // 2
    assert acc.argmax() == c * cfg.fft_m + c
    # point symmetry of the PSF of a real field about (M/2, M/2)
    inner = acc[1:, 1:]
    assert np.abs(inner - inner[::-1, ::-1]).max() < 1e-5


def test_accumulates_into_existing_values(torch_dev):
    cfg = G.PsfConfig(pupil_n=64, pupil_dx_m=39.0 / 64)
    opd = _opd(2, 64, 0.3)
    base = torch_dev.full((cfg.fft_m, cfg.fft_m), 0.25, device="cuda")
    acc, _ = run_gpu(torch_dev, cfg, opd, acc0=base)
    want, _ = OP.psf_accumulate(cfg, opd)
    assert np.abs(acc - 0.25 - want).max() <= TOL * want.max()


def test_zero_frames_noop_and_bad_arguments(torch_dev):
    import ctypes as C

    from paper_1408_0698_amd import shwfs
    cfg = G.PsfConfig(pupil_n=64, pupil_dx_m=39.0 / 64)
    plan = _plan(cfg)
    acc = torch_dev.zeros((cfg.fft_m, cfg.fft_m), device="cuda")
    plan.accumulate(torch_dev.zeros((0, 64, 64), device="cuda"), acc)
    torch_dev.cuda.synchronize()
    assert float(acc.abs().max()) == 0.0
    d = torch_dev.zeros((1, 64, 64), device="cuda")
    assert shwfs._lib.psf_accumulate(plan._h, C.c_void_p(d.data_ptr()), 63, 0, 1, C.c_void_p(acc.data_ptr()),
                                     None, None) == shwfs.E_INVALID
    assert shwfs._lib.psf_accumulate(plan._h, C.c_void_p(d.data_ptr()), 64, -5, 1, C.c_void_p(acc.data_ptr()),
                                     None, None) == shwfs.E_INVALID


def test_star_batch_equals_single_calls(torch_dev):
    """3 stars x 5 frames in one call: every star equals its own call, bitwise; one star vs the oracle."""
    cfg = G.PsfConfig(pupil_n=160, pupil_dx_m=39.0 / 160)
    opd = np.stack([_opd(5, 160, 0.1, seed=s) for s in (1, 2, 3)])
    plan = _plan(cfg)
    d = torch_dev.from_numpy(opd).cuda()
    acc = torch_dev.zeros((3, 1600, 1600), device="cuda")
    sr = torch_dev.zeros((3, 5), device="cuda")
    plan.accumulate_stars(d, acc, sr)
    torch_dev.cuda.synchronize()
    for s in range(3):
        a1, s1 = run_gpu(torch_dev, cfg, opd[s])
        assert np.array_equal(acc[s].cpu().numpy(), a1.astype(np.float32))
        assert np.array_equal(sr[s].cpu().numpy(), s1.astype(np.float32))
    want, want_sr = OP.psf_accumulate(cfg, opd[1])
    assert np.abs(acc[1].cpu().numpy() - want).max() <= TOL * want.max()
    assert np.abs(sr[1].cpu().numpy() - want_sr).max() <= TOL * want_sr.max()


def test_unaligned_accumulators_equal_aligned(torch_dev):
    """Accumulators at a 4-byte offset, with a star stride that is not a multiple of 4 floats (the
    column pass then updates them 4 bytes at a time): bitwise the same sums as 16-byte aligned ones."""
    cfg = G.PsfConfig(pupil_n=96, pupil_dx_m=39.0 / 96)
    m = cfg.fft_m
    opd = np.stack([_opd(2, 96, 0.2, seed=s) for s in (4, 5)])
    plan = _plan(cfg)
    d = torch_dev.from_numpy(opd).cuda()
    aligned = torch_dev.full((2, m, m), 0.5, device="cuda")
    plan.accumulate_stars(d, aligned)
    stride = m * m + 3
    buf = torch_dev.full((1 + 2 * stride,), 0.5, device="cuda")
    odd = buf[1:].as_strided((2, m, m), (stride, m, 1))
    plan.accumulate_stars(d, odd)
    torch_dev.cuda.synchronize()
    assert np.array_equal(odd.cpu().numpy(), aligned.cpu().numpy())
    # the floats between the two accumulators are untouched
    assert np.all(buf[1 + m * m:1 + stride].cpu().numpy() == 0.5)
    want, _ = OP.psf_accumulate(cfg, opd[0])
    assert np.abs(aligned[0].cpu().numpy() - 0.5 - want).max() <= TOL * want.max()
