"""FP64 CPU oracle for the Shack-Hartmann measurement and the science PSF.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct definition that the GPU path is checked against.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and it shares no code with
the HIP kernels.

Every transform is an explicit DFT matrix product (no FFT algorithm).
Each function cites the passage of the paper it follows:

* Sec. 4, "LGS Shack Hartmann wavefront sensor": split the wavefront into
  sub-apertures, spot by Fourier transform per sub-aperture, elongation
  by convolution with a Gaussian, noise, centroid -> slopes.
* Sec. 3, closed-loop block: X- and Y-slope vectors from the residual
  phase (open-loop wavefront minus the DM).
* Sec. 3, PSF block: PSF at the chosen wavelength(s) weighted by the object's
  colour, Strehl ratio and encircled energy.
* Sec. 4, open-loop generation: screens piled up per direction, the cone
  effect of finite-altitude sources and the LGS uplink tip-tilt.
* Sec. 2: the 800x800 pupil at 4.875e-2 m/px and the ~5000/1400/1800 DM modes.

The paper prints no equations, so each formula is a reading; the readings
are listed in ``READINGS`` and in the design notes.  Parts with no anchor
outside this package (the physical realism of the LGS spot) are "parity
unpinned": only self-consistency with the readings is checked.
"""
from . import geometry, philox, wfs, psf, dm, calib, loop, openloop  # noqa: F401

READINGS = {
    "O1": "binary pupil, pixel-centre test, linear obstruction ratio",
    "O2": "valid sub-aperture iff illuminated fraction >= min_illum; row-major order",
    "O3": "half-pixel centred DFT, exp(-2 pi i ...) forward sign, I = |F|^2 / N^2",
    "O4": "FFT pixel = lambda / (fft_n dx); detector pixel = (conv_n / det_n) FFT pixels",
    "O5": "elongated Gaussian, hexagonal edge launchers, periodised on a symmetric lattice",
    "O6": "circular convolution by DFT multiply",
    "O7": "area-overlap rebin",
    "O8": "photometry scaled by illuminated fraction; Philox4x32-10 pair blocks: Poisson + read noise",
    "O9": "thresholded centre of gravity, zero slopes and a flag when nothing is left",
    "O11": "fftshift-centred PSF normalised by (sum A)^2; Strehl = on-axis sample",
    "O12": "Gaussian influence functions, integer-pixel DM and screen shifts",
    "O13": "sodium sub-layers: point-source wavefront of each beam height against the focus height",
    "O14": "closed loop: actuator modes, coefs += gain * CM s, push-pull columns (s+ - s-) / 2a",
    "O15": "cone effect: layer sampled at (1 - h/H) r + h theta, bilinear; uplink tilt = LS tilt over the launch beam",
    "O16": "polychromatic PSF: PSFs resampled bilinearly to the reference wavelength's grid and weighted; EE in pixels",
}
