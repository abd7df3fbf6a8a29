"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test states what fixes the expected value independently of the
oracle's own code, so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

from gen import configs as C
from oracle import dm as D
from oracle import geometry as G
from oracle import philox as P
from oracle import psf as PS
from oracle import wfs as O

RNG = np.random.default_rng(12345)


def dirichlet2(t, n, N):
    """sin^2(pi n t / N) / sin^2(pi t / N), with its limit n^2 at integer multiples of N."""
    t = np.asarray(t, dtype=np.float64)
    den = np.sin(np.pi * t / N) ** 2
    near = np.abs(den) < 1e-300
    return np.where(near, float(n * n), np.sin(np.pi * n * t / N) ** 2 / np.where(near, 1.0, den))


def _cfg(**kw):
    base = dict(pupil_n=8, pupil_dx_m=0.1, obstruction=0.0, n_subap=2, min_illum=0.5, fft_n=8,
                conv_n=8, wavelength_m=0.5e-6, lgs=0, det_n=8)
    base.update(kw)
    return C.WfsConfig(**base)


# ---------------------------------------------------------------- O1 / O2 geometry

def test_pupil_area_matches_annulus_area():
    # pixel count of a sampled annulus approaches pi/4 N^2 (1 - eps^2)
    for n, tol in ((80, 2.0), (800, 20.0)):
        area = math.pi / 4 * n * n * (1 - 0.14 ** 2)
        assert abs(G.pupil_mask(n, 0.14).sum() - area) < tol


def test_pupil_is_symmetric_and_obstructed():
    A = G.pupil_mask(80, 0.14)
    assert np.array_equal(A, A[::-1, :]) and np.array_equal(A, A.T)
    assert A[40, 40] == 0 and A[40, 0] == 1 and A[0, 0] == 0


def test_valid_subaps_by_counting():
    # brute-force count of lit pixels per sub-aperture with explicit loops
    cfg = C.CFG0
    A = G.pupil_mask(cfg.pupil_n, cfg.obstruction)
    n = cfg.npx
    want = []
    for a in range(cfg.n_subap):
        for b in range(cfg.n_subap):
            lit = sum(A[a * n + i, b * n + j] for i in range(n) for j in range(n))
            if 2 * lit >= n * n:
                want.append(a * cfg.n_subap + b)
    vi, il = G.subap_table(cfg)
    assert list(vi) == want and len(vi) == 80
    assert np.all(il >= 0.5) and np.all(il <= 1.0)


# ---------------------------------------------------------------- O3 spot

def _brute_spot(e, N):
    n = e.shape[0]
    c = (N - 1) / 2
    I = np.zeros((N, N))
    for v in range(N):
        for u in range(N):
            s = 0j
            for y in range(n):
                for x in range(n):
                    s += e[y, x] * np.exp(-2j * np.pi * ((u - c) * x + (v - c) * y) / N)
            I[v, u] = abs(s) ** 2 / N ** 2
    return I


@pytest.mark.parametrize("n,N", [(2, 4), (3, 6), (4, 8), (3, 8)])
def test_spot_equals_bruteforce_dft(n, N):
    e = RNG.standard_normal((n, n)) * np.exp(1j * RNG.uniform(0, 2 * np.pi, (n, n)))
    cfg = _cfg(fft_n=N)
    I = O.spot_intensity(cfg, e[None])[0]
    assert np.max(np.abs(I - _brute_spot(e, N))) < 1e-12 * max(1.0, np.abs(I).max())


def test_parseval():
    A = (RNG.uniform(size=(10, 10)) > 0.3).astype(float)
    e = A * np.exp(1j * RNG.normal(0, 3, (10, 10)))
    I = O.spot_intensity(_cfg(fft_n=40), e[None])[0]
    assert abs(I.sum() - (A ** 2).sum()) < 1e-10


@pytest.mark.parametrize("n,N", [(8, 16), (10, 40), (10, 20)])
def test_square_subap_is_dirichlet_squared(n, N):
    # flat, fully lit n x n square: I(v,u) = D(u-c) D(v-c) / N^2, D = sin^2(pi n t/N)/sin^2(pi t/N)
    c = (N - 1) / 2
    Dt = dirichlet2(np.arange(N) - c, n, N)
    I = O.spot_intensity(_cfg(fft_n=N), np.ones((1, n, n), complex))[0]
    assert np.max(np.abs(I - np.outer(Dt, Dt) / N ** 2)) < 1e-11 * I.max()


def _kernel_khat(N, sp, sq, psi):
    return G.kernel_spectrum(G.sodium_kernel(N, sp, sq, psi)).real


@pytest.mark.parametrize("conv", [False, True])
def test_flat_wavefront_any_real_amplitude_gives_zero_slopes(conv):
    # Hermitian symmetry of a real field's transform: the spot is point-symmetric about (c, c),
    # for any real amplitude, any rebin factor (here 2.5) and a point-symmetric kernel.
    A = RNG.uniform(-1, 1, (4, 10, 10))
    I = O.spot_intensity(_cfg(fft_n=40), A.astype(complex))
    if conv:
        K = np.stack([_kernel_khat(40, 7.0, 2.0, 0.7), _kernel_khat(40, 3.0, 3.0, 0.0),
                      _kernel_khat(40, 15.0, 1.5, -2.1), _kernel_khat(40, 4.0, 2.0, 1.3)])
        I = O.convolve(I, K)
    det = O.rebin(I, 16)
    sx, sy, empty = O.centroid(det, 0.0)
    assert not empty.any()
    assert np.max(np.abs(sx)) < 1e-12 and np.max(np.abs(sy)) < 1e-12


@pytest.mark.parametrize("n,N,s", [(8, 16, 0.1), (8, 16, 0.5), (8, 16, 1.0), (8, 16, 2.0),
                                   (10, 40, 0.1), (10, 40, 1.0), (10, 40, -3.3)])
def test_tilt_centroid_matches_windowed_dirichlet(n, N, s):
    # phase 2 pi s x / N on a full square: I(v,u) = D(v-c) D(u-c-s) / N^2 and the
    # centroid (one FFT pixel per detector pixel) is sum (u-c) D(u-c-s) / sum D(u-c-s)
    c = (N - 1) / 2
    x = np.arange(n)
    e = np.exp(2j * np.pi * s * x[None, :] / N) * np.ones((n, 1))
    I = O.spot_intensity(_cfg(fft_n=N), e[None])
    sx, sy, _ = O.centroid(I, 0.0)
    Dt = dirichlet2(np.arange(N) - c - s, n, N)
    want = ((np.arange(N) - c) * Dt).sum() / Dt.sum()
    assert abs(sx[0] - want) < 1e-10 and abs(sy[0]) < 1e-12


def test_half_pixel_tilt_is_exact():
    n, N = 8, 16
    e = np.exp(2j * np.pi * 0.5 * np.arange(n)[None, :] / N) * np.ones((n, 1))
    sx, _, _ = O.centroid(O.spot_intensity(_cfg(fft_n=N), e[None]), 0.0)
    assert abs(sx[0] - 0.5) < 1e-12


@pytest.mark.parametrize("s", [1, 3, -2])
def test_integer_tilt_is_circular_shift(s):
    A = (RNG.uniform(size=(10, 10)) > 0.2).astype(float)
    ph = RNG.normal(0, 1, (10, 10))
    N = 40
    x = np.arange(10)[None, :]
    e0 = A * np.exp(1j * ph)
    e1 = e0 * np.exp(2j * np.pi * s * x / N)
    I0 = O.spot_intensity(_cfg(fft_n=N), e0[None])[0]
    I1 = O.spot_intensity(_cfg(fft_n=N), e1[None])[0]
    assert np.max(np.abs(I1 - np.roll(I0, s, axis=1))) < 1e-10


# ---------------------------------------------------------------- O5 / O6 kernel and convolution

@pytest.mark.parametrize("sp,sq,psi", [(3.0, 3.0, 0.0), (20.7, 3.4, 2.2), (8.0, 1.0, -0.4)])
def test_kernel_normalised_symmetric_real_spectrum(sp, sq, psi):
    k = G.sodium_kernel(40, sp, sq, psi)
    assert abs(k.sum() - 1) < 1e-14
    # point symmetry about (0, 0) on the circular grid
    kr = np.roll(k[::-1, ::-1], (1, 1), axis=(0, 1))
    assert np.max(np.abs(k - kr)) < 1e-17 * 40
    K = G.kernel_spectrum(k)
    assert np.max(np.abs(K.imag)) < 1e-12
    assert abs(K[0, 0].real - 1) < 1e-13


def test_kernel_long_axis_follows_psi():
    # second moments of the kernel: the long axis lies along (cos psi, sin psi)
    k = G.sodium_kernel(40, 4.0, 1.0, math.pi / 6)
    t = np.arange(40)
    t = np.where(t <= 20, t, t - 40).astype(float)
    mxx = (k * t[None, :] ** 2).sum()
    myy = (k * t[:, None] ** 2).sum()
    mxy = (k * t[None, :] * t[:, None]).sum()
    ang = 0.5 * math.atan2(2 * mxy, mxx - myy)
    assert abs(ang - math.pi / 6) < 1e-3
    assert abs(mxx + myy - (16 + 1)) < 1e-3


def test_narrow_kernel_is_identity():
    K = _kernel_khat(40, 0.05, 0.05, 0.3)
    assert np.max(np.abs(K - 1)) < 1e-12


def test_convolution_equals_bruteforce_circular_sum():
    N = 8
    I = RNG.uniform(size=(N, N))
    k = G.sodium_kernel(N, 1.7, 0.6, 0.9)
    want = np.zeros((N, N))
    for v in range(N):
        for u in range(N):
            want[v, u] = sum(I[i, j] * k[(v - i) % N, (u - j) % N] for i in range(N) for j in range(N))
    J = O.convolve(I[None], G.kernel_spectrum(k).real[None])[0]
    assert np.max(np.abs(J - want)) < 1e-13
    assert abs(J.sum() - I.sum()) < 1e-12


def test_elongation_geometry():
    cfg = C.CFG1
    launch = C.launch_positions(cfg, 6)
    vi, _ = G.subap_table(cfg)
    sp, sq, psi = G.elongation_params(cfg, launch[0], vi)
    px = G.fft_pixel_rad(cfg) / G.ARCSEC
    f = 1 / (2 * math.sqrt(2 * math.log(2)))
    assert np.allclose(sq, 0.5 * f / px)
    # capped law: 0..3 arcsec over the diameter, added in quadrature to 0.5 arcsec
    assert sp.max() * px / f < math.sqrt(3.0 ** 2 + 0.25) and sp.max() * px / f > 2.9
    # the sub-aperture nearest the launcher (at +x edge) is nearly round; psi points away from it
    i = np.argmin(sp)
    xs, ys = G.subap_centres_m(cfg, vi)
    assert xs[i] > 18.0 and abs(ys[i]) < 0.5
    far = np.nonzero(xs == xs.min())[0]
    j = far[np.argmin(np.abs(ys[far]))]   # far side, on the launcher's axis
    assert abs(abs(psi[j]) - math.pi) < 0.01


# ---------------------------------------------------------------- O4 plate scale, O5 widths in arcsec
# The angular size of an FFT pixel is measured here from what a wavefront tilt does to the spot,
# through the oracle's field formation and transform only; no plate-scale formula is used.  A plane
# wave arriving at angle theta adds OPD = x sin(theta) across the pupil.  The spot of an n-sample
# field zero-padded to N >= 2n is a trigonometric polynomial of degree < n in the pixel index, so a
# tilt moves it by an exact, generally fractional, shift s, and its DFT along that axis at frequency
# k takes the factor exp(-2 pi i k s / N).

def _tilt_shift_px(cfg, theta_rad, axis, sel=(0, 1000, 2500, 4000)):
    """Spot shift in FFT pixels caused by an OPD tilt of theta along x (axis 1) or y (axis 0)."""
    vi, _ = G.subap_table(cfg)
    vi = vi[list(sel)]
    rng = np.random.default_rng(41)
    base = rng.normal(0.0, 0.2 * cfg.wavelength_m, (cfg.pupil_n, cfg.pupil_n))
    coord = (np.arange(cfg.pupil_n) + 0.5 - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    tilt = np.sin(theta_rad) * (coord[None, :] if axis == 1 else coord[:, None])
    N = cfg.fft_n
    n = cfg.pupil_n // cfg.n_subap
    I0 = O.spot_intensity(cfg, O.subap_fields(cfg, base, vi))
    I1 = O.spot_intensity(cfg, O.subap_fields(cfg, base + tilt, vi))
    F0 = np.fft.fft(I0, axis=1 + axis)
    F1 = np.fft.fft(I1, axis=1 + axis)
    k1 = (slice(None), slice(None), 1) if axis == 1 else (slice(None), 1, slice(None))
    s = -np.angle(np.sum(F1[k1] * np.conj(F0[k1]))) * N / (2 * np.pi)
    # the shift is exact at every in-band frequency, not only at k = 1
    k = np.arange(N)
    kk = np.where(k < N / 2, k, k - N)
    ph = np.exp(-2j * np.pi * kk * s / N)
    band = np.abs(kk) < n
    shape = (1, 1, N) if axis == 1 else (1, N, 1)
    want = F0 * ph.reshape(shape)
    sl = (slice(None), slice(None), band) if axis == 1 else (slice(None), band, slice(None))
    assert np.abs(F1[sl] - want[sl]).max() < 1e-9 * np.abs(F0).max()
    return s


@pytest.mark.parametrize("cfg_name", ["CFG0", "CFG1", "CFG1_R2"])
@pytest.mark.parametrize("axis", [1, 0])
def test_fft_pixel_angle_from_the_tilt_response(cfg_name, axis):
    cfg = getattr(C, cfg_name).replace(lgs=0)
    theta = 0.37 * G.ARCSEC
    sel = (0, 30, 55, 79) if cfg.n_subap == 10 else (0, 1000, 2500, 4000)
    s = _tilt_shift_px(cfg, theta, axis, sel)
    assert s > 0  # a positive tilt moves the spot to larger pixel indices (reading O3)
    assert abs(s * G.fft_pixel_rad(cfg) - theta) < 1e-9 * theta
    assert abs(G.det_pixel_rad(cfg) / G.fft_pixel_rad(cfg) - cfg.conv_n / cfg.det_n) < 1e-15


def _fwhm_arcsec_from_spectrum(khat_axis_1, N, px_rad):
    """FWHM of a Gaussian kernel from its DFT at frequency 1 along one axis.

    The DFT of the periodised samples of exp(-t^2 / 2 sigma^2) at integer frequency k is exactly the
    continuous transform there, exp(-2 pi^2 sigma^2 k^2 / N^2), up to the aliasing of the sampling
    (negligible for sigma >= 1 px); a Gaussian falls to half its peak at sigma sqrt(2 ln 2).
    """
    sigma_px = N * math.sqrt(-math.log(khat_axis_1) / 2.0) / math.pi
    return 2.0 * sigma_px * math.sqrt(2.0 * math.log(2.0)) * px_rad / G.ARCSEC


@pytest.mark.parametrize("frac", [1.0 / 3.0, 0.1, 0.55])
def test_elongated_kernel_widths_in_arcsec(frac):
    """The kernel of a sub-aperture at distance d from its launcher has FWHM sqrt((3'' d/D)^2 + 0.5''^2)
    along the launcher direction and 0.5'' across it (reading O5), in angles measured by the tilt."""
    cfg = C.CFG1
    theta = 0.37 * G.ARCSEC
    px = theta / _tilt_shift_px(cfg.replace(lgs=0), theta, 1)
    vi, _ = G.subap_table(cfg)
    i = 1234
    n = cfg.pupil_n // cfg.n_subap
    a, b = divmod(int(vi[i]), cfg.n_subap)
    xc = ((b + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    yc = ((a + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    D = cfg.pupil_n * cfg.pupil_dx_m
    d = frac * D
    K = O.kernel_spectra(cfg, (xc - d, yc), vi[[i]])[0]   # launcher on the -x side: long axis along x
    par = _fwhm_arcsec_from_spectrum(K[0, 1], cfg.conv_n, px)
    perp = _fwhm_arcsec_from_spectrum(K[1, 0], cfg.conv_n, px)
    assert abs(par - math.hypot(3.0 * frac, 0.5)) < 1e-6
    assert abs(perp - 0.5) < 1e-6


def test_geometric_elongation_law_in_arcsec():
    """elong_max <= 0: the elongation is the sodium layer's depth seen from a distance d, d * dh / H^2."""
    cfg = C.CFG1.replace(elong_max_arcsec=0.0)
    theta = 0.37 * G.ARCSEC
    px = theta / _tilt_shift_px(cfg.replace(lgs=0), theta, 0)
    vi, _ = G.subap_table(cfg)
    i = 777
    n = cfg.pupil_n // cfg.n_subap
    a, b = divmod(int(vi[i]), cfg.n_subap)
    xc = ((b + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    yc = ((a + 0.5) * n - cfg.pupil_n / 2.0) * cfg.pupil_dx_m
    d = 3.0
    K = O.kernel_spectra(cfg, (xc, yc - d), vi[[i]])[0]   # launcher on the -y side: long axis along y
    el = d * 10e3 / 90e3 ** 2 / G.ARCSEC
    assert abs(_fwhm_arcsec_from_spectrum(K[1, 0], cfg.conv_n, px) - math.hypot(el, 0.5)) < 1e-6
    assert abs(_fwhm_arcsec_from_spectrum(K[0, 1], cfg.conv_n, px) - 0.5) < 1e-6


def test_round_laser_spot_kernel_in_arcsec():
    """The sub-layer form's kernel is the round 0.5'' laser spot, in angles measured by the tilt."""
    cfg = C.CFG1
    theta = 0.37 * G.ARCSEC
    px = theta / _tilt_shift_px(cfg.replace(lgs=0), theta, 1)
    K = O.round_kernel_spectrum(cfg)
    for v in (K[0, 1], K[1, 0]):
        assert abs(_fwhm_arcsec_from_spectrum(v, cfg.conv_n, px) - 0.5) < 1e-6


# ---------------------------------------------------------------- O7 rebin

@pytest.mark.parametrize("N,d", [(40, 16), (16, 8), (512, 16), (40, 40)])
def test_rebin_weights(N, d):
    W = O.rebin_matrix(N, d)
    assert np.allclose(W.sum(axis=1), N / d) and np.allclose(W.sum(axis=0), 1.0)
    J = RNG.uniform(size=(1, N, N))
    assert abs(O.rebin(J, d).sum() - J.sum()) < 1e-9


def test_integer_rebin_is_block_sum():
    J = RNG.uniform(size=(1, 16, 16))
    want = J[0].reshape(8, 2, 8, 2).sum(axis=(1, 3))
    assert np.max(np.abs(O.rebin(J, 8)[0] - want)) < 1e-14


def test_fractional_rebin_pattern():
    W = O.rebin_matrix(40, 16)
    assert np.allclose(W[0, :4], [1, 1, 0.5, 0]) and np.allclose(W[1, 2:6], [0.5, 1, 1, 0])


# ---------------------------------------------------------------- O8 noise

def test_philox_known_answers(golden_dir):
    for line in open(os.path.join(golden_dir, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        out = P.philox4x32_10(*[np.array([c], np.uint64) for c in v[:4]], v[4], v[5])
        assert [int(o[0]) for o in out] == v[6:]


def test_uniform_is_exact_and_open():
    x = np.array([0, 511, 512, 0xFFFFFFFF], np.uint32)
    u = P.uniform_f32(x)
    assert u.dtype == np.float32
    assert u[0] == np.float32(2.0 ** -24) and u[1] == u[0]
    assert u[3] == np.float32(1 - 2.0 ** -24) and u[3] < 1


def _poisson_sample(lam, n, seed=77):
    # one image of n pixels: pixels b and b + n/2 share a pair block
    pix = np.arange(n, dtype=np.uint64)
    return P.poisson_counts(np.full(n, lam, np.float32), seed, pix, 5, 9, n)


@pytest.mark.parametrize("lam", [0.3, 2.5, 9.5, 10.0, 19.7, 20.0, 31.7, 250.0])
def test_poisson_moments_and_pmf(lam):
    n = 400_000
    k = _poisson_sample(lam, n)
    assert abs(k.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(k.var() / lam - 1) < 5 * math.sqrt(2.0 / n) + 0.01
    # chi-square against the Poisson pmf over bins with >= 50 expected
    ks = np.arange(int(lam + 12 * math.sqrt(lam) + 12))
    pmf = np.exp(-lam + ks * math.log(lam) - np.array([math.lgamma(v + 1) for v in ks]))
    obs = np.bincount(k, minlength=len(ks))[: len(ks)]
    exp = pmf * n
    m = exp >= 50
    chi2 = (((obs[m] - exp[m]) ** 2) / exp[m]).sum()
    dof = m.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    # the two pixels of a pair block draw independent counts (words 0 and 1, or their own trials)
    h = n // 2
    r = np.corrcoef(k[:h].astype(np.float64), k[h:].astype(np.float64))[0, 1]
    assert abs(r) < 5 / math.sqrt(h)


def test_poisson_inversion_small_uniform_gives_zero():
    assert P.poisson_inversion_f32(np.float32(3.0), np.float32(1e-3)) == 0
    # u just above e^-lam moves to 1
    lam = np.float32(2.0)
    e = float(np.exp(-lam))
    assert P.poisson_inversion_f32(lam, np.float32(e * 1.01)) == 1


def test_inversion_matches_fp64_search_away_from_ties():
    rng = np.random.default_rng(3)
    # the whole range the inversion serves: 0 < lambda < POISSON_SPLIT (= 20)
    lam = rng.uniform(0.1, P.POISSON_SPLIT, 20000).astype(np.float32)
    lam = np.minimum(lam, np.nextafter(np.float32(P.POISSON_SPLIT), np.float32(0)))
    u = P.uniform_f32(rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32))
    k32 = P.poisson_inversion_f32(lam, u)
    assert (lam[:4000] >= 10.0).sum() > 1500
    for l, uu, k in zip(lam[:4000], u[:4000], k32[:4000]):
        F, p, kk = math.exp(-float(l)), math.exp(-float(l)), 0
        while float(uu) > F:
            kk += 1
            p *= float(l) / kk
            F += p
        assert kk == k or P.inversion_margin(l, uu) < 1e-6


def test_read_noise_unit_variance():
    n = 300_000
    z = P.read_noise(11, np.arange(n, dtype=np.uint64), 2, 4, n)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert abs(np.mean(z ** 4) - 3) < 0.05
    # both deviates of a Box-Muller pair: each standard normal, uncorrelated, and uncorrelated in
    # their squares (r cos and r sin of one draw are independent)
    h = n // 2
    c, s_ = z[:h], z[h:]
    for half in (c, s_):
        assert abs(half.mean()) < 0.015 and abs(half.var() - 1) < 0.015
    assert abs(np.corrcoef(c, s_)[0, 1]) < 5 / math.sqrt(h)
    assert abs(np.corrcoef(c ** 2, s_ ** 2)[0, 1]) < 5 / math.sqrt(h)


def test_pair_block_assignment():
    # n = 5 pixels: h = 3; pixels (0, 3) and (1, 4) share blocks 0 and 1, pixel 2 has block 2 alone
    pix = np.arange(5, dtype=np.uint64)
    w, second = P.pair_block(21, pix, 5, 7, 3)
    assert list(second) == [False, False, False, True, True]
    w0 = P.noise_words(21, np.zeros(3, np.uint64), np.arange(3, dtype=np.uint64), 7, 3)
    for i, b in enumerate([0, 1, 2, 0, 1]):
        assert all(int(w[j][i]) == int(w0[j][b]) for j in range(4))
    z = P.read_noise(21, pix, 7, 3, 5)
    r = np.sqrt(-2.0 * np.log(P.uniform_f32(w0[2]).astype(np.float64)))
    th = 2.0 * np.pi * P.uniform_f32(w0[3]).astype(np.float64)
    assert np.allclose(z[:3] ** 2 + np.r_[z[3:], 0.0] ** 2, r ** 2 * np.r_[1.0, 1.0, np.cos(th[2]) ** 2])


def test_noise_counters_are_independent_of_batching():
    lam = np.full((3, 4, 4), 5.0, np.float32)
    a = P.poisson_counts(lam, 9, np.arange(16, dtype=np.uint64).reshape(1, 4, 4),
                         np.arange(3, dtype=np.uint64).reshape(3, 1, 1), 2, 16)
    b = P.poisson_counts(lam[1:2], 9, np.arange(16, dtype=np.uint64).reshape(1, 4, 4),
                         np.array([1], np.uint64).reshape(1, 1, 1), 2, 16)
    assert np.array_equal(a[1:2], b)


# ---------------------------------------------------------------- O9 centroid

def test_single_pixel_centroid():
    img = np.zeros((1, 16, 16))
    img[0, 3, 11] = 7.0
    sx, sy, e = O.centroid(img, 0.0)
    assert sx[0] == 11 - 7.5 and sy[0] == 3 - 7.5 and not e[0]


def test_threshold_above_max_flags_empty():
    img = RNG.uniform(0, 1, (2, 8, 8))
    sx, sy, e = O.centroid(img, 1.5)
    assert e.all() and np.all(sx == 0) and np.all(sy == 0)


def test_threshold_subtracts_before_weighting():
    img = np.zeros((1, 4, 4))
    img[0, 0, 0] = 4.0
    img[0, 0, 3] = 2.0
    sx, _, _ = O.centroid(img, 1.0)
    assert abs(sx[0] - (3 * (-1.5) + 1 * 1.5) / 4) < 1e-15


# ---------------------------------------------------------------- whole-pipeline brute force

def test_tiny_lgs_pipeline_bruteforce():
    """Every step by explicit loops on a tiny LGS geometry (pupil 8, 2x2 sub-apertures)."""
    cfg = _cfg(pupil_n=8, n_subap=2, fft_n=8, conv_n=8, det_n=4, lgs=1, obstruction=0.2,
               photons_per_subap=100.0, elong_max_arcsec=0.4, spot_fwhm_arcsec=0.1)
    launch = [(0.4, 0.0)]
    opd = (RNG.normal(0, 0.2e-6, (8, 8))).astype(np.float32)
    sens = O.Sensor(cfg, 1, launch)
    got = sens.measure(opd[None, None])
    A = G.pupil_mask(8, 0.2)
    vi, il = G.subap_table(cfg)
    sp, sq, psi = G.elongation_params(cfg, launch[0], vi)
    for s, idx in enumerate(vi):
        a, b = divmod(int(idx), 2)
        e = np.array([[A[a * 4 + y, b * 4 + x] * np.exp(2j * np.pi * float(opd[a * 4 + y, b * 4 + x]) / 0.5e-6)
                       for x in range(4)] for y in range(4)])
        I = _brute_spot(e, 8)
        k = G.sodium_kernel(8, sp[s], sq[s], psi[s])
        J = np.zeros((8, 8))
        for v in range(8):
            for u in range(8):
                J[v, u] = sum(I[i, j] * k[(v - i) % 8, (u - j) % 8] for i in range(8) for j in range(8))
        det = np.zeros((4, 4))
        for p in range(4):
            for q in range(4):
                det[p, q] = J[2 * p:2 * p + 2, 2 * q:2 * q + 2].sum()
        img = 100.0 * il[s] * det / det.sum()
        cx = sum((q - 1.5) * img[p, q] for p in range(4) for q in range(4)) / img.sum()
        cy = sum((p - 1.5) * img[p, q] for p in range(4) for q in range(4)) / img.sum()
        assert np.max(np.abs(got["images"][0, 0, s] - img)) < 1e-12 * img.max()
        assert abs(got["slopes"][0, 0, 0, s] - cx) < 1e-12 and abs(got["slopes"][0, 0, 1, s] - cy) < 1e-12


# ---------------------------------------------------------------- O11 PSF

def test_psf_tiny_bruteforce_and_strehl():
    cfg = C.PsfConfig(pupil_n=6, pupil_dx_m=0.1, obstruction=0.0, fft_m=12, wavelength_m=1e-6)
    A = G.pupil_mask(6, 0.0)
    opd = RNG.normal(0, 0.1e-6, (6, 6))
    P1 = PS.psf_frame(cfg, opd)
    e = A * np.exp(2j * np.pi * opd / 1e-6)
    want = np.zeros((12, 12))
    for v in range(12):
        for u in range(12):
            s = sum(e[y, x] * np.exp(-2j * np.pi * ((u - 6) * x + (v - 6) * y) / 12)
                    for y in range(6) for x in range(6))
            want[v, u] = abs(s) ** 2 / A.sum() ** 2
    assert np.max(np.abs(P1 - want)) < 1e-13
    assert abs(P1[6, 6] - PS.strehl_direct(cfg, opd)) < 1e-14


def test_psf_flat_piston_parseval():
    cfg = C.PsfConfig(pupil_n=40, pupil_dx_m=0.2, obstruction=0.14, fft_m=80, wavelength_m=1.65e-6)
    A = G.pupil_mask(40, 0.14)
    P0 = PS.psf_frame(cfg, np.zeros((40, 40)))
    assert abs(P0[40, 40] - 1) < 1e-13
    opd = RNG.normal(0, 0.2e-6, (40, 40))
    P1 = PS.psf_frame(cfg, opd)
    P2 = PS.psf_frame(cfg, opd + 0.37e-6)
    assert np.max(np.abs(P1 - P2)) < 1e-13
    assert abs(P1.sum() - 80 * 80 / A.sum()) < 1e-9
    acc, sr = PS.psf_accumulate(cfg, [opd, np.zeros((40, 40))])
    assert abs(sr[1] - 1) < 1e-13 and np.allclose(acc, P1 + P0)


# ---------------------------------------------------------------- O12 DM

def test_actuator_counts_match_paper_mode_counts():
    n = [len(D.actuators(800, 4.875e-2, h, p, 60.0)) for h, p in C.DMS]
    assert n == [5025, 1413, 1781]
    # Sec. 2 quotes ~5000, ~1400 and ~1800 modes
    assert abs(n[0] - 5000) < 50 and abs(n[1] - 1400) < 50 and abs(n[2] - 1800) < 50
    assert [D.surface_size(800, 4.875e-2, h, 60.0) for h, _ in C.DMS] == [800, 848, 952]


def test_influence_function_coupling():
    s = D.dm_surface(100, np.array([[0.0, 0.0], [10.0, 0.0]]), [1.0, 0.0], 10)
    # actuator 0 sits at the pixel corner (50, 50): the four nearest centres are 0.5 px away
    v_center = s[49:51, 49:51].mean()
    v_pitch = s[49:51, 59:61].mean()
    sig = D.influence_sigma(10, 0.3)
    assert abs(v_center - math.exp(-0.5 / (2 * sig * sig))) < 1e-12
    r2 = 9.5 ** 2 + 0.5 ** 2
    assert abs(s[50, 59] - math.exp(-r2 / (2 * sig * sig))) < 1e-12
    assert abs(math.exp(-100 / (2 * sig * sig)) - 0.3) < 1e-12
    assert s.sum() > 0 and np.count_nonzero(s) == 64 * 64


def test_residual_is_screen_minus_shifted_surfaces():
    scr = RNG.normal(size=(30, 30))
    s1 = RNG.normal(size=(12, 12))
    out = D.residual_opd(scr, (2, 5), [s1], [(1, 3)], 8)
    assert np.array_equal(out, scr[2:10, 5:13] - s1[1:9, 3:11])
    assert D.footprint_shift_px(12700, 60, 4.875e-2) == 76 and D.footprint_shift_px(4000, -60, 4.875e-2) == -24


# ---------------------------------------------------------------- O13 sodium sub-layers

def _sodium_cfg(ns=2, **kw):
    return C.CFG1.replace(pupil_n=10 * ns, n_subap=ns, obstruction=0.0, flags=0, photons_per_subap=0.0,
                          threshold_e=0.0, **kw)


@pytest.mark.parametrize("dh", [-2000.0, 1500.0])
def test_sublayer_opd_gradient_is_parallax_angle(dh):
    """The OPD slope equals the change of the exact 3-D direction to the beam point between heights H + dh and H."""
    cfg = _sodium_cfg(13)
    L = (6.1, -2.3)
    opd = O.sublayer_opd(cfg, L, dh)
    dx = cfg.pupil_dx_m
    H = cfg.na_height_m
    for (i, j) in [(3, 4), (60, 100), (120, 7)]:
        x = (j + 0.5 - cfg.pupil_n / 2) * dx
        y = (i + 0.5 - cfg.pupil_n / 2) * dx

        def cosines(h):
            v = np.array([L[0] - x, L[1] - y, h])
            return v[:2] / np.linalg.norm(v)
        want = cosines(H + dh) - cosines(H)
        gx = (opd[i, j + 1] - opd[i, j - 1]) / (2 * dx)
        gy = (opd[i + 1, j] - opd[i - 1, j]) / (2 * dx)
        assert abs(gx - want[0]) < 1e-5 * abs(want[0]) and abs(gy - want[1]) < 1e-5 * abs(want[1])


@pytest.mark.parametrize("s", [2, -3])
def test_sublayer_integer_parallax_is_circular_shift(s):
    """A launcher placed so that the sub-layer tilt over a sub-aperture is s FFT pixels shifts the spot by s
    against the launcher at the sub-aperture centre (same defocus in both)."""
    cfg = _sodium_cfg(2)
    valid, _ = G.subap_table(cfg)
    dh = -2000.0
    H = cfg.na_height_m
    kappa = 1.0 / (H + dh) - 1.0 / H
    rc = ((0.5 * 10) - cfg.pupil_n / 2) * cfg.pupil_dx_m          # sub-aperture 0 centre, x and y
    shift = s * cfg.wavelength_m / (cfg.fft_n * cfg.pupil_dx_m * kappa)
    at_c = O.spot_intensity(cfg, O.subap_fields(cfg, O.sublayer_opd(cfg, (rc, rc), dh), valid[:1]))[0]
    off = O.spot_intensity(cfg, O.subap_fields(cfg, O.sublayer_opd(cfg, (rc + shift, rc), dh), valid[:1]))[0]
    assert np.abs(off - np.roll(at_c, s, axis=1)).max() < 1e-9 * at_c.max()
    assert np.abs(at_c - at_c.T).max() < 1e-9 * at_c.max()      # pure defocus: symmetric in x and y


def test_sodium_single_layer_at_focus_is_the_round_kernel_form():
    cfg = _sodium_cfg(4)
    L = [(1.0, -0.5)]
    opd = np.random.default_rng(3).normal(0, 2e-7, (1, 1, 40, 40))
    a = O.Sensor(cfg, 1, L, sodium=([0.0], [1.0])).measure(opd)
    b = O.Sensor(cfg.replace(elong_max_arcsec=1e-12), 1, L).measure(opd)
    assert np.abs(a["images"] - b["images"]).max() < 1e-12 * np.abs(b["images"]).max()


def test_sodium_weights_are_normalised():
    cfg = _sodium_cfg(3)
    L = [(0.5, 0.7)]
    opd = np.zeros((1, 1, 30, 30))
    a = O.Sensor(cfg, 1, L, sodium=([-1500.0, 0.0, 1500.0], [1.0, 2.0, 1.0])).measure(opd)
    b = O.Sensor(cfg, 1, L, sodium=([-1500.0, 0.0, 1500.0], [0.25, 0.5, 0.25])).measure(opd)
    assert np.abs(a["images"] - b["images"]).max() < 1e-14


def test_sodium_elongation_axis_points_from_launcher():
    """Flat wavefront, three equal sub-layers: the spot's long axis is the launcher-to-sub-aperture direction."""
    cfg = _sodium_cfg(20, spot_fwhm_arcsec=0.2)
    D = cfg.diameter_m
    L = [(D / 2, 0.0)]
    sens = O.Sensor(cfg, 1, L, sodium=([-3000.0, 0.0, 3000.0], [1.0, 1.0, 1.0]))
    valid = sens.valid_idx
    xs, ys = G.subap_centres_m(cfg, valid)
    pick = [int(np.argmin(np.hypot(xs - px, ys - py))) for (px, py) in [(-3.0, 3.0), (0.0, -4.0), (-4.5, 0.0)]]
    r = sens.measure(np.zeros((1, 1, cfg.pupil_n, cfg.pupil_n)), subset=pick)
    d = cfg.det_n
    q = np.arange(d) - (d - 1) / 2
    for k, i in enumerate(pick):
        img = r["images"][0, 0, k]
        m = img.sum()
        cx = (img * q[None, :]).sum() / m
        cy = (img * q[:, None]).sum() / m
        cxx = (img * (q[None, :] - cx) ** 2).sum() / m
        cyy = (img * (q[:, None] - cy) ** 2).sum() / m
        cxy = (img * (q[None, :] - cx) * (q[:, None] - cy)).sum() / m
        axis = 0.5 * math.atan2(2 * cxy, cxx - cyy)
        psi = math.atan2(ys[i] - L[0][1], xs[i] - L[0][0])
        diff = (axis - psi + math.pi / 2) % math.pi - math.pi / 2
        assert abs(diff) < math.radians(3.0), (i, math.degrees(axis), math.degrees(psi))
        assert cxx + cyy > 0


# ---------------------------------------------------------------- O15 cone effect and uplink tilt

from oracle import openloop as OL  # noqa: E402


def _plane(rows, cols, a, b, c):
    X, Y = np.meshgrid(np.arange(cols, dtype=np.float64), np.arange(rows, dtype=np.float64))
    return a + b * X + c * Y


def test_projection_of_a_plane_is_the_plane_at_the_cone_footprint():
    # bilinear interpolation reproduces a plane exactly, so the projection is a closed form
    N, dx = 24, 0.5
    layers = [(_plane(200, 220, 1e-7, 2e-9, -3e-9), 0.25, 0.0, 110.3, 99.7),
              (_plane(300, 300, -2e-7, 5e-9, 1e-9), 0.5, 8000.0, 150.0, 149.5)]
    theta, H = (3e-5, -2e-5), 90000.0
    got = OL.project(layers, N, dx, theta, H)
    x, y = OL.pupil_coords(N, dx)
    want = np.zeros_like(x)
    for S, p, h, x0, y0 in layers:
        s = 1 - h / H
        X = x0 + (s * x + h * theta[0]) / p
        Y = y0 + (s * y + h * theta[1]) / p
        a, b, c = S[0, 0], S[0, 1] - S[0, 0], S[1, 0] - S[0, 0]
        want += a + b * X + c * Y
    assert np.abs(got - want).max() < 1e-18


def test_projection_ground_layer_integer_origin_is_a_window():
    # h = 0 and pupil pixel centres on integer screen samples: the OPD is a plain window
    rng = np.random.default_rng(4)
    S = rng.normal(size=(64, 64))
    N, dx = 16, 1.0
    got = OL.project([(S, 1.0, 0.0, 20.5 + N / 2 - 0.5 + 0.5, 10.0 + N / 2)], N, dx, (0.0, 0.0), 0.0)
    # pixel j centre x = j + 1/2 - N/2 -> X = 20.5 + N/2 + (j + 1/2 - N/2) = 21 + j; Y = 10 + N/2 + y = 10.5 + i
    X0, Y0 = 21.0, 10.5
    assert X0 == int(X0)
    want_rows = 0.5 * (S[10:10 + N, 21:21 + N] + S[11:11 + N, 21:21 + N])
    assert np.allclose(got, want_rows, rtol=0, atol=1e-15)


def test_cone_shrinks_the_footprint_by_one_minus_h_over_H():
    # a plane of slope b per metre on a layer at h seen by a source at H = 2h has slope b / 2
    N, dx, h = 20, 0.5, 5000.0
    layer = (_plane(100, 100, 0.0, 1e-8, 0.0), 0.5, h, 50.0, 50.0)
    near = OL.project([layer], N, dx, (0.0, 0.0), 2 * h)
    far = OL.project([layer], N, dx, (0.0, 0.0), 0.0)
    assert np.allclose(np.diff(near, axis=1), 0.5 * np.diff(far, axis=1), rtol=1e-12, atol=0)


def test_uplink_tilt_of_planes_and_quadratics():
    # least squares over a symmetric sample set: a plane gives its slope, a quadratic the slope at the centre
    pitch = 0.1
    lay = [(_plane(400, 400, 3e-7, 4e-9, -1e-9), pitch, 0.0, 200.0, 200.0),
           (_plane(400, 400, 0.0, -2e-9, 6e-9), pitch, 6000.0, 200.0, 200.0)]
    tx, ty = OL.uplink_tilt(lay, (10.0, -5.0), (2e-5, 1e-5), 90000.0, 0.4, 32)
    assert abs(tx - (4e-9 - 2e-9) / pitch) < 1e-18 and abs(ty - (-1e-9 + 6e-9) / pitch) < 1e-18
    X, Y = np.meshgrid(np.arange(400.0), np.arange(400.0))
    q = 1e-9 * ((X - 180.0) ** 2 + 0.5 * (Y - 230.0) ** 2)   # gradient (2 (X - 180), (Y - 230)) e-9 per sample
    lx, ly = 3.0, -2.0                                         # beam centre at (200 + 30, 200 - 20) samples, h = 0
    tx, ty = OL.uplink_tilt([(q, pitch, 0.0, 200.0, 200.0)], (lx, ly), (0.0, 0.0), 90000.0, 0.4, 40)
    # bilinear interpolation of a quadratic adds a periodic error; its LS slope over the beam is small
    assert abs(tx - 2e-9 * (230.0 - 180.0) / pitch) < 2e-3 * abs(2e-9 * 50 / pitch)
    assert abs(ty - 1e-9 * (180.0 - 230.0) / pitch) < 2e-3 * abs(1e-9 * 50 / pitch)


# ---------------------------------------------------------------- O16 encircled energy, polychromatic PSF

from oracle import psf as OPSF  # noqa: E402
from gen.configs import PsfConfig  # noqa: E402


def test_encircled_energy_matches_the_airy_closed_form():
    cfg = PsfConfig(pupil_n=64, pupil_dx_m=0.1, obstruction=0.0, fft_m=512, wavelength_m=1e-6)
    acc, _ = OPSF.psf_accumulate(cfg, [np.zeros((64, 64))])
    r = np.array([4.0, 8.0, 12.0, 20.0, 40.0])   # lambda/D is 8 px
    ee = OPSF.encircled_energy(acc, r)
    want = OPSF.airy_encircled_energy(r, 64, 512)
    # pixelated pupil, pixelated radii and the periodic M grid: agreement to ~1 %
    assert np.abs(ee - want).max() < 0.015
    assert np.all(np.diff(ee) > 0)
    assert OPSF.encircled_energy(acc, [1e9])[0] == 1.0
    assert OPSF.encircled_energy(acc, [0.0])[0] == acc[256, 256] / acc.sum()


def test_resample_identity_and_scaled_gaussian():
    rng = np.random.default_rng(8)
    P = rng.random((32, 32))
    assert np.array_equal(OPSF.resample(P, 1.0), P)
    # a wide Gaussian: resampling by s reads it at s times the distance from the centre
    M, c = 128, 64
    d = np.arange(M, dtype=np.float64) - c
    G = np.exp(-(d[None, :] ** 2 + d[:, None] ** 2) / (2 * 15.0 ** 2))
    Q = OPSF.resample(G, 0.8)
    want = np.exp(-((0.8 * d[None, :]) ** 2 + (0.8 * d[:, None]) ** 2) / (2 * 15.0 ** 2))
    assert np.abs(Q - want).max() < 2e-3


def test_polychromatic_strehl_of_a_flat_wavefront_is_the_weight_sum():
    base = PsfConfig(pupil_n=32, pupil_dx_m=0.1, obstruction=0.14, fft_m=128, wavelength_m=1.65e-6)
    cfgs = [base, base.__class__(**{**base.__dict__, "wavelength_m": 1.5e-6}),
            base.__class__(**{**base.__dict__, "wavelength_m": 1.8e-6})]
    w = [0.5, 0.2, 0.3]
    P = OPSF.polychromatic(cfgs, w, [np.zeros((32, 32))])
    assert abs(P[64, 64] - sum(w)) < 1e-12


def test_inversion_never_runs_to_the_cap_where_the_fp32_cdf_saturates():
    # for these means the FP32 cumulative sum ends a few 1e-7 below the largest uniform; the search
    # stops where the sum stops growing, at a count consistent with the mean, not at the step cap
    u = np.float32(1 - 2.0 ** -24)
    for lam in (0.01189812, 0.0200900, 0.0536567, 3.3, 9.7, 15.5, 19.9):
        lam = np.float32(lam)
        k = int(P.poisson_inversion_f32(lam, u))
        assert k < P.INVERSION_MAX_K
        assert k <= lam + 12 * math.sqrt(lam) + 12
        # the probability of k or more, in FP64, is far below the uniform's resolution
        tail = 1.0 - sum(math.exp(-float(lam)) * float(lam) ** j / math.factorial(j) for j in range(k))
        assert tail < 1e-6
