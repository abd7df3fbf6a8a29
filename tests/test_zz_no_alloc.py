"""The allocation-free encircled-energy entry point (static device workspace) against the
allocating one, through the C ABI: bitwise-equal results on two calls in a row, the second with
fewer PSFs and fewer radii, and host-side rejection of requests beyond the static workspace.
Inputs are seeded on the host."""
import numpy as np
import pytest

from gen import configs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _psfs(M, n, seed):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:M, 0:M].astype(np.float64) - M / 2
    out = []
    for s in range(n):
        w = rng.uniform(3.0, 40.0)
        core = np.exp(-((x - rng.uniform(-2, 2)) ** 2 + (y - rng.uniform(-2, 2)) ** 2) / (2 * w * w))
        out.append((core + 1e-4 * rng.random((M, M))).astype(np.float32))
    return np.stack(out)


def test_noalloc_matches_allocating_entry_point(torch_dev):
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    cfg = G.CFG3
    print("no-alloc encircled energy: M", cfg.fft_m, flush=True)
    plan = shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, cfg.fft_m, cfg.wavelength_m)
    # first call: 7 PSFs at 40 radii; second: 3 other PSFs at 11 radii (smaller in both)
    for n_psf, radii, seed in ((7, [0.5 + 9.7 * k for k in range(40)], 11), (3, [0.0, 1.0, 2.5, 4.0, 8.0, 16.0,
                                                                                    33.3, 64.0, 300.0, 799.0, 5000.0], 12)):
        print(f"  call with {n_psf} PSFs, {len(radii)} radii", flush=True)
        P = torch.from_numpy(_psfs(cfg.fft_m, n_psf, seed)).cuda()
        got = torch.full((n_psf, len(radii)), -1.0, dtype=torch.float64, device="cuda")
        plan.encircled_energy(P, radii, out=got, noalloc=True)
        want = plan.encircled_energy(P, radii)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(g, w), np.abs(g - w).max()
        assert np.all((g >= 0) & (g <= 1))
    plan.close()


def test_noalloc_rejects_requests_beyond_the_static_workspace(torch_dev):
    """Host-side rejection.  The buffers are real and large enough for every access the kernels
    would make, so the call is safe whatever the check decides."""
    from paper_1408_0698_amd import shwfs
    torch = torch_dev
    cfg = G.CFG3
    M, n_psf, n_r = cfg.fft_m, 41, 64
    assert n_psf * 200 * (n_r + 1) > 2 ** 19          # 533,000 doubles: one PSF too many
    assert (n_psf - 1) * 200 * (n_r + 1) <= 2 ** 19   # 520,000: fits
    print("no-alloc rejection: M", M, n_psf, "PSFs,", n_r, "radii", flush=True)
    plan = shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, M, cfg.wavelength_m)
    gen = torch.Generator(device="cuda").manual_seed(13)
    P = torch.rand((n_psf, M, M), generator=gen, device="cuda")
    radii = [0.5 * k for k in range(n_r)]
    out = torch.zeros((n_psf, n_r), dtype=torch.float64, device="cuda")
    with pytest.raises(shwfs.ShwError) as ei:
        plan.encircled_energy(P, radii, out=out, noalloc=True)
    assert ei.value.code == shwfs.E_INVALID and "static workspace" in str(ei.value)
    # one PSF fewer fits and equals the allocating entry point
    got = plan.encircled_energy(P[:-1], radii, out=out[:-1], noalloc=True)
    want = plan.encircled_energy(P[:-1], radii)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())
    plan.close()
