"""The band-limited inverse column transform + column rebin of the fused kernel (csrc/band_rebin.h:
pixel pairs as shifts, one 8-point inverse transform for both phases), compiled for the host and
checked against its definition in FP64: the real inverse DFT of a Hermitian spectrum that is zero
outside the band, then the area-overlap rebin (the oracle's rebin weights, reading O7).  No GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import wfs as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1408_0698_amd", "csrc")
N, DN, NB = 40, 16, 10   # the 39 m LGS shape: conv_n 40, 16 detector pixels, 10-pixel sub-apertures
CASES = 6

PROGRAM = r"""
#include "band_rebin.h"
#include <cstdio>
#include <cstdlib>
using namespace shw;
int main(int argc, char** argv) {
  // spectra from argv: CASES x (NB real parts, NB imaginary parts)
  int a = 1;
  for (int c = 0; c < %(cases)d; ++c) {
    float zr[%(nb)d], zi[%(nb)d], col[%(n)d];
    for (int k = 0; k < %(nb)d; ++k) zr[k] = std::strtof(argv[a++], nullptr);
    for (int k = 0; k < %(nb)d; ++k) zi[k] = std::strtof(argv[a++], nullptr);
    band_rebin_column<%(n)d, %(dn)d, %(nb)d>(zr, zi, col);
    for (int p = 0; p < %(dn)d; ++p) std::printf("%%.9e ", col[p]);
    std::printf("\n");
  }
  return 0;
}
""" % {"cases": CASES, "nb": NB, "n": N, "dn": DN}


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_band_rebin_map_is_inverse_transform_then_rebin(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    rng = np.random.default_rng(1408)
    spectra = []
    for c in range(CASES):
        zr = rng.normal(size=NB).astype(np.float32)
        zi = rng.normal(size=NB).astype(np.float32)
        zi[0] = 0.0
        if c == 0:          # a single lag: one cosine across the column
            zr[:] = 0.0
            zi[:] = 0.0
            zr[3] = 1.0
        spectra.append((zr, zi))
    src, exe = tmp_path / "band_rebin_host.cpp", tmp_path / "band_rebin_host"
    src.write_text(PROGRAM)
    r = subprocess.run([hipcc, "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    args = [f"{v:.9e}" for zr, zi in spectra for v in list(zr) + list(zi)]
    out = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=60, check=True).stdout
    got = np.array([[float(t) for t in line.split()] for line in out.strip().splitlines()])
    assert got.shape == (CASES, DN)
    wr = W.rebin_matrix(N, DN)   # area-overlap weights, rows sum to N / DN
    u = np.arange(N)
    for c, (zr, zi) in enumerate(spectra):
        R = np.zeros(N, complex)
        R[:NB] = zr.astype(np.float64) + 1j * zi.astype(np.float64)
        R[N - NB + 1:] = np.conj(R[1:NB][::-1])      # Hermitian: the column is real
        J = np.array([(R * np.exp(2j * np.pi * uu * np.arange(N) / N)).sum() for uu in u])
        assert np.abs(J.imag).max() < 1e-9
        ref = wr @ J.real
        scale = np.abs(wr) @ np.abs(J.real) + 1e-30
        assert np.abs(got[c] - ref).max() <= 2e-6 * scale.max(), c
