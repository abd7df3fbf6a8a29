"""Oracle Shack-Hartmann measurement (FP64, explicit DFT matrices).

Test infrastructure (see the package docstring).

Follows the LGS Shack-Hartmann module of Sec. 4: the wavefront is split
into sub-apertures, the spot of each is computed by Fourier transform,
the spot is convolved with a Gaussian for the physical extent of the
laser projection on the sodium layer, noise is added, and the centroid of
the final image gives the slopes; the slope vector is X then Y
(Sec. 3, closed-loop block).  The step order below is that order.
"""
from __future__ import annotations

import numpy as np

from . import geometry as G
from . import philox as P


def centred_dft(N: int, n: int) -> np.ndarray:
    """W[u, x] = exp(-2 pi i (u - c) x / N), c = (N-1)/2, x < n (reading O3).

    The half-pixel centre makes the spot of a real field point-symmetric
    about (c, c); the forward sign puts a positive phase gradient at a
    positive pixel offset.
    """
    c = (N - 1) / 2.0
    u = np.arange(N, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    return np.exp(-2j * np.pi * (u - c) * x / N)


def subap_fields(cfg, opd_m, valid_idx):
    """Complex field A exp(2 pi i OPD / lambda) of each valid sub-aperture.

    opd_m: [pupil_n][pupil_n] OPD in metres.  Returns [S][n][n] complex.
    """
    A = G.pupil_mask(cfg.pupil_n, cfg.obstruction)
    n = cfg.pupil_n // cfg.n_subap
    opd = np.asarray(opd_m, dtype=np.float64)
    a = valid_idx // cfg.n_subap
    b = valid_idx % cfg.n_subap
    rows = a[:, None, None] * n + np.arange(n)[None, :, None]
    cols = b[:, None, None] * n + np.arange(n)[None, None, :]
    phi = 2.0 * np.pi * opd[rows, cols] / cfg.wavelength_m
    return A[rows, cols] * np.exp(1j * phi)


def spot_intensity(cfg, fields):
    """I = |W e W^T|^2 / N^2 per sub-aperture (reading O3): [S][fft_n][fft_n]."""
    N = cfg.fft_n
    W = centred_dft(N, fields.shape[-1])
    F = W[None] @ fields @ W.T[None]
    return (F.real ** 2 + F.imag ** 2) / float(N * N)


def embed(cfg, I):
    """Place the fft_n spot at offset (conv_n - fft_n)/2 of the conv_n grid."""
    if cfg.conv_n == cfg.fft_n:
        return I
    o = (cfg.conv_n - cfg.fft_n) // 2
    out = np.zeros(I.shape[:-2] + (cfg.conv_n, cfg.conv_n))
    out[..., o:o + cfg.fft_n, o:o + cfg.fft_n] = I
    return out


def kernel_spectra(cfg, launch_xy, valid_idx):
    """Real K^ of every valid sub-aperture for one launcher: [S][conv_n][conv_n]."""
    sp, sq, psi = G.elongation_params(cfg, launch_xy, valid_idx)
    out = np.empty((len(valid_idx), cfg.conv_n, cfg.conv_n))
    for i in range(len(valid_idx)):
        k = G.sodium_kernel(cfg.conv_n, sp[i], sq[i], psi[i])
        out[i] = G.kernel_spectrum(k).real
    return out


def convolve(I, Khat):
    """J = Re IDFT2(DFT2(I) K^), the circular convolution of I with k (reading O6)."""
    N = I.shape[-1]
    F = G.dft_matrix(N)
    X = F[None] @ I @ F.T[None]
    Y = X * Khat
    Fi = np.conj(F)
    return (Fi[None] @ Y @ Fi.T[None]).real / float(N * N)


def rebin_matrix(conv_n: int, det_n: int) -> np.ndarray:
    """W[p, k] = overlap of [k, k+1) with [b p, b (p+1)), b = conv_n / det_n (reading O7)."""
    b = conv_n / det_n
    p = np.arange(det_n, dtype=np.float64)[:, None]
    k = np.arange(conv_n, dtype=np.float64)[None, :]
    return np.maximum(0.0, np.minimum(k + 1.0, b * (p + 1.0)) - np.maximum(k, b * p))


def rebin(J, det_n):
    W = rebin_matrix(J.shape[-1], det_n)
    return W[None] @ J @ W.T[None]


def photometry(cfg, det, illum):
    """Expected electrons: n_ph * f * Det / sum Det (reading O8); Det itself when n_ph = 0."""
    if cfg.photons_per_subap <= 0:
        return det
    tot = det.sum(axis=(-1, -2), keepdims=True)
    tot = np.where(tot > 0, tot, 1.0)
    return cfg.photons_per_subap * illum[:, None, None] * det / tot


def add_noise(cfg, lam, seed, gsub, frame):
    """Poisson counts plus read noise (Sec. 4 noise-added image; reading O8)."""
    S, d, _ = lam.shape
    pix = np.arange(d * d, dtype=np.uint64).reshape(1, d, d)
    g = np.asarray(gsub, dtype=np.uint64).reshape(S, 1, 1)
    counts = P.poisson_counts(lam.astype(np.float32), seed, pix, g, np.uint64(frame), d * d)
    z = P.read_noise(seed, pix, g, np.uint64(frame), d * d)
    return counts.astype(np.float64) + cfg.ron_e * z, counts


def centroid(img, threshold):
    """Thresholded centre of gravity in detector pixels from the centre (reading O9).

    Returns (sx, sy, empty): sx along columns, sy along rows; sub-apertures
    with nothing above threshold get (0, 0) and empty = True.
    """
    d = img.shape[-1]
    It = np.maximum(img - threshold, 0.0)
    c = (d - 1) / 2.0
    q = np.arange(d, dtype=np.float64) - c
    tot = It.sum(axis=(-1, -2))
    sx_num = (It * q[None, None, :]).sum(axis=(-1, -2))
    sy_num = (It * q[None, :, None]).sum(axis=(-1, -2))
    empty = tot <= 0
    safe = np.where(empty, 1.0, tot)
    return np.where(empty, 0.0, sx_num / safe), np.where(empty, 0.0, sy_num / safe), empty


def sublayer_opd(cfg, launch_xy, dh_m):
    """Extra OPD (metres) over the pupil for the sodium sub-layer at height H + dh (reading O13).

    Sec. 4: each sodium sub-layer brings its own tip-tilt and defocus.  The
    beam point at height h above the launcher at L is a point source; its
    spherical wavefront at pupil point r, taken against the one from the
    focus height H, is -|r - L|^2 / 2 * (1/h - 1/H) (paraxial).
    """
    n = cfg.pupil_n
    c = (np.arange(n, dtype=np.float64) + 0.5 - n / 2.0) * cfg.pupil_dx_m
    x = c[None, :] - launch_xy[0]
    y = c[:, None] - launch_xy[1]
    H = cfg.na_height_m
    return -0.5 * (x * x + y * y) * (1.0 / (H + dh_m) - 1.0 / H)


def round_kernel_spectrum(cfg):
    """K^ of the round laser spot (FWHM spot_fwhm_arcsec) on the conv grid: the sub-layer form's kernel."""
    px_as = G.fft_pixel_rad(cfg) / G.ARCSEC
    sigma = cfg.spot_fwhm_arcsec / (2.0 * np.sqrt(2.0 * np.log(2.0))) / px_as
    return G.kernel_spectrum(G.sodium_kernel(cfg.conv_n, sigma, sigma, 0.0)).real


def measure_one(cfg, opd_m, valid_idx, illum, khat=None, seed=0, gsub0=0, frame=0,
                chunk=2048, subset=None, layers=None):
    """One sensor, one frame.  Returns dict(slopes=[2][S], images=[S][d][d], empty=[S]).

    khat: callable mapping sub-aperture indices to their K^ (LGS only).

    subset: optional indices into valid_idx to evaluate only some sub-apertures
    (their global ids and noise counters stay those of the full sensor).

    layers: optional list of (weight, opd) for the sodium sub-layer form: the
    spot is sum_j weight_j |transform of sub-layer j|^2 (Sec. 4: per-sub-layer
    spots times the profile, piled up) and opd_m is not used.
    """
    sel = np.arange(len(valid_idx)) if subset is None else np.asarray(subset)
    noise = bool(cfg.flags & 1) and cfg.photons_per_subap > 0
    thr = cfg.threshold_e if cfg.photons_per_subap > 0 else 0.0
    imgs = np.empty((len(sel), cfg.det_n, cfg.det_n))
    lams = np.empty((len(sel), cfg.det_n, cfg.det_n))
    sx = np.empty(len(sel))
    sy = np.empty(len(sel))
    empty = np.empty(len(sel), dtype=bool)
    for s0 in range(0, len(sel), chunk):
        ii = sel[s0:s0 + chunk]
        if layers is None:
            I = spot_intensity(cfg, subap_fields(cfg, opd_m, valid_idx[ii]))
        else:
            I = sum(wt * spot_intensity(cfg, subap_fields(cfg, o, valid_idx[ii])) for wt, o in layers)
        I = embed(cfg, I)
        J = convolve(I, khat(ii)) if cfg.lgs else I
        det = rebin(J, cfg.det_n)
        lam = photometry(cfg, det, illum[ii])
        if noise:
            img, _ = add_noise(cfg, lam, seed, gsub0 + ii, frame)
        else:
            img = lam
        x, y, e = centroid(img, thr)
        imgs[s0:s0 + len(ii)] = img
        lams[s0:s0 + len(ii)] = lam
        sx[s0:s0 + len(ii)] = x
        sy[s0:s0 + len(ii)] = y
        empty[s0:s0 + len(ii)] = e
    return dict(slopes=np.stack([sx, sy]), images=imgs, lam=lams, empty=empty)


class Sensor:
    """n_wfs sensors of one geometry: tables built once (plan setup, Sec. 4 inputs)."""

    def __init__(self, cfg, n_wfs=1, launch=None, sodium=None):
        """sodium: optional (dh_m, weight): the sodium sub-layer form (weights normalised to unit sum)."""
        self.cfg = cfg
        self.n_wfs = n_wfs
        self.valid_idx, self.illum = G.subap_table(cfg)
        self.n_valid = len(self.valid_idx)
        self.launch = launch
        self._khat = {}
        self.sodium = None
        if sodium is not None:
            dh = np.asarray(sodium[0], dtype=np.float64)
            wt = np.asarray(sodium[1], dtype=np.float64)
            self.sodium = (dh, wt / wt.sum())
            self._round = round_kernel_spectrum(cfg)
            self._sub_opd = [[sublayer_opd(cfg, launch[w], d) for d in dh] for w in range(n_wfs)]

    def khat(self, w, sel):
        """K^ of sub-apertures sel of sensor w ([len(sel)][conv_n][conv_n]), cached."""
        if not self.cfg.lgs:
            return None
        if self.sodium is not None:
            return np.broadcast_to(self._round, (len(sel),) + self._round.shape)
        need = [int(i) for i in sel if (w, int(i)) not in self._khat]
        if need:
            ks = kernel_spectra(self.cfg, self.launch[w], self.valid_idx[need])
            for i, k in zip(need, ks):
                self._khat[(w, i)] = k
        return np.stack([self._khat[(w, int(i))] for i in sel])

    def measure(self, opd, seed=0, frame0=0, subset=None):
        """opd: [n_frames][n_wfs][N_p][N_p], or [n_frames][n_wfs][n_sub][N_p][N_p] for the sub-layer form.

        Returns slopes [F][W][2][S'], images [F][W][S'][d][d] (electrons after noise),
        lam (expected electrons before noise, same shape) and empty [F][W][S'].
        """
        opd = np.asarray(opd)
        nf = opd.shape[0]
        S = self.n_valid if subset is None else len(subset)
        slopes = np.empty((nf, self.n_wfs, 2, S))
        images = np.empty((nf, self.n_wfs, S, self.cfg.det_n, self.cfg.det_n))
        lam = np.empty_like(images)
        empty = np.empty((nf, self.n_wfs, S), dtype=bool)
        for f in range(nf):
            for w in range(self.n_wfs):
                layers = None
                if self.sodium is not None:
                    dh, wt = self.sodium
                    per_layer = opd.ndim == 5
                    layers = [(wt[j], np.asarray(opd[f, w, j] if per_layer else opd[f, w], dtype=np.float64)
                               + self._sub_opd[w][j]) for j in range(len(dh))]
                r = measure_one(self.cfg, opd[f, w], self.valid_idx, self.illum,
                                (lambda ii, w=w: self.khat(w, ii)),
                                seed=seed, gsub0=w * self.n_valid, frame=frame0 + f, subset=subset, layers=layers)
                slopes[f, w] = r["slopes"]
                images[f, w] = r["images"]
                lam[f, w] = r["lam"]
                empty[f, w] = r["empty"]
        return dict(slopes=slopes, images=images, lam=lam, empty=empty)
