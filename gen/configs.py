"""Workload parameters for the five synthetic workloads.

This module holds numbers only: it computes nothing of the sensor model.
Both the FP64 oracle and the GPU path read these values; each derives its
own geometry (pupil, valid sub-apertures, kernels) independently.

Field meanings follow the problem statement of the LGS Shack-Hartmann
module (paper Sec. 4, "LGS Shack Hartmann wavefront sensor") and the
telescope sampling of paper Sec. 2 (800x800 pupil at 4.875e-2 m/px).
"""
from __future__ import annotations

import dataclasses
import math

ARCSEC = math.pi / (180.0 * 3600.0)

FLAG_NOISE = 1
FLAG_RETURN_IMAGES = 2
# precision selector, bits 4..7
PREC_FP32 = 0
PREC_BF16 = 1
PREC_BF16X3 = 2
PREC_FP16X3 = 3


@dataclasses.dataclass(frozen=True)
class WfsConfig:
    """One Shack-Hartmann sensor geometry (shared by n_wfs sensors)."""

    pupil_n: int                 # pupil sampling, pixels across
    pupil_dx_m: float            # metres per pupil pixel
    obstruction: float           # linear central obstruction ratio
    n_subap: int                 # sub-apertures across the pupil
    min_illum: float             # valid if illuminated fraction >= this
    fft_n: int                   # spot FFT size (zero padded)
    conv_n: int                  # convolution grid (>= fft_n)
    wavelength_m: float
    lgs: int                     # 0 = NGS (no sodium kernel)
    na_height_m: float = 90e3
    na_fwhm_m: float = 10e3
    elong_max_arcsec: float = 3.0    # <= 0: geometric law d*fwhm/H^2
    spot_fwhm_arcsec: float = 0.5    # laser spot on the sodium layer
    det_n: int = 8
    photons_per_subap: float = 0.0   # 0: no photometry and no noise
    ron_e: float = 0.0
    threshold_e: float = 0.0
    flags: int = 0

    @property
    def npx(self) -> int:
        return self.pupil_n // self.n_subap

    @property
    def diameter_m(self) -> float:
        return self.pupil_n * self.pupil_dx_m

    def replace(self, **kw) -> "WfsConfig":
        return dataclasses.replace(self, **kw)


def launch_positions(cfg: WfsConfig, n_wfs: int):
    """Launch telescope positions (x, y) in metres, one per sensor.

    Six launchers on the pupil edge, hexagonally spaced (a reading of
    "launch from pupil edge").  Returned as plain numbers: both sides
    take them as inputs.
    """
    r = cfg.diameter_m / 2.0
    return [(r * math.cos(math.radians(60.0 * w)), r * math.sin(math.radians(60.0 * w)))
            for w in range(n_wfs)]


# 8 m telescope, one NGS SH-WFS, noise off.
CFG0 = WfsConfig(pupil_n=80, pupil_dx_m=0.1, obstruction=0.14, n_subap=10, min_illum=0.5,
                 fft_n=16, conv_n=16, wavelength_m=0.75e-6, lgs=0, det_n=8)

# 39 m pupil, LGS, 80x80 sub-apertures of 10x10 px, FFT 40 (2x oversampled beyond the
# Nyquist size 20), 16x16 detector pixels, 500 photons and 3 e- read noise.
CFG1 = WfsConfig(pupil_n=800, pupil_dx_m=4.875e-2, obstruction=0.14, n_subap=80, min_illum=0.5,
                 fft_n=40, conv_n=40, wavelength_m=589e-9, lgs=1, na_height_m=90e3,
                 na_fwhm_m=10e3, elong_max_arcsec=3.0, spot_fwhm_arcsec=0.5, det_n=16,
                 photons_per_subap=500.0, ron_e=3.0, threshold_e=3.0, flags=FLAG_NOISE)
CFG1_NWFS = 6

# The alternative reading of "padded to 20x20 (then 2x oversampled 40x40)": spot FFT 20,
# intensity embedded in a 40x40 convolution grid.
CFG1_R2 = CFG1.replace(fft_n=20, conv_n=40)

# Sodium sub-layer form of the 39 m LGS sensor: three sub-layers (the count of the paper's
# timing).  The profile is a Gaussian of FWHM t cut into n equal slabs over [-t, t], each
# sub-layer at its slab centre with the slab's share of the profile as weight.  t is the
# thickness whose geometric elongation across the diameter, t D / H^2, equals the
# elongation of the single-kernel form (3 arcsec), so the two forms see the same spread.
def sodium_profile(n_sub: int, thickness_m: float):
    """(dh_m, weight) of n_sub slabs of a Gaussian profile of FWHM thickness_m over [-t, t]."""
    sigma = thickness_m / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    edges = [-thickness_m + 2.0 * thickness_m * k / n_sub for k in range(n_sub + 1)]
    cdf = [0.5 * (1.0 + math.erf(e / (sigma * math.sqrt(2.0)))) for e in edges]
    dh = [0.5 * (edges[k] + edges[k + 1]) for k in range(n_sub)]
    wt = [cdf[k + 1] - cdf[k] for k in range(n_sub)]
    tot = sum(wt)
    return dh, [v / tot for v in wt]


SODIUM_NSUB = 3
SODIUM_THICKNESS_M = (CFG1.elong_max_arcsec * math.pi / (180.0 * 3600.0)) * CFG1.na_height_m ** 2 / CFG1.diameter_m
SODIUM = sodium_profile(SODIUM_NSUB, SODIUM_THICKNESS_M)

# cfg4 NGS: 2x2 sub-apertures of 400x400 px padded to 512, detector 16x16.
CFG4_NGS = WfsConfig(pupil_n=800, pupil_dx_m=4.875e-2, obstruction=0.14, n_subap=2, min_illum=0.5,
                     fft_n=512, conv_n=512, wavelength_m=0.75e-6, lgs=0, det_n=16,
                     photons_per_subap=500.0, ron_e=3.0, threshold_e=3.0, flags=FLAG_NOISE)
CFG4_NNGS = 3


@dataclasses.dataclass(frozen=True)
class PsfConfig:
    pupil_n: int = 800
    pupil_dx_m: float = 4.875e-2
    obstruction: float = 0.14
    fft_m: int = 1600
    wavelength_m: float = 1.65e-6     # H band


CFG3 = PsfConfig()
# 3x3 test stars over 2x2 arcmin (offsets in arcsec).
CFG3_STARS = [(tx, ty) for ty in (-60.0, 0.0, 60.0) for tx in (-60.0, 0.0, 60.0)]
CFG3_FRAMES = 20

# Deformable mirrors for the residual: (altitude m, pitch px).  The post-focal altitudes
# are assumed (the paper gives none); with a 60 arcsec field radius they give
# 1413 and 1781 actuators, matching the ~1400 and ~1800 modes of the paper.
DMS = [(0.0, 10), (4000.0, 20), (12700.0, 20)]
DM_FIELD_RADIUS_ARCSEC = 60.0
DM_PATCH = 64
DM_COUPLING = 0.3
DM_COEF_RMS_M = 50e-9

# Screens: von Karman at 0.5 um.
SCREEN_R0_M = 0.15
SCREEN_L0_M = 25.0
SCREEN_LAMBDA0_M = 0.5e-6
SCREEN_SEED = 1408
NOISE_SEED = 698
