"""The register FFTs of the kernels (csrc/regfft.h), compiled for the host and checked against the
DFT definition in FP64: the prime-factor lengths (10, 20, 40, 80: no twiddles between the two sets
of short transforms) and the Cooley-Tukey ones (8, 16, 32), both directions.  No GPU needed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1408_0698_amd", "csrc")
SIZES = (5, 8, 10, 16, 20, 32, 40, 80)

PROGRAM = r"""
#include "regfft.h"
#include <cmath>
#include <cstdio>
using namespace shw;
template <int N, int DIR> void run() {
  float2 x[N];
  for (int i = 0; i < N; ++i) x[i] = make_float2((float)std::sin(1.3 * i + 0.2), (float)std::cos(0.7 * i * i + 0.1));
  RegFFT<N, DIR>::run(x);
  std::printf("%d %d", N, DIR);
  for (int i = 0; i < N; ++i) std::printf(" %.9e %.9e", x[i].x, x[i].y);
  std::printf("\n");
}
int main() {
  run<5, -1>(); run<8, -1>(); run<10, -1>(); run<16, -1>(); run<20, -1>(); run<32, -1>(); run<40, -1>(); run<80, -1>();
  run<5, 1>(); run<8, 1>(); run<10, 1>(); run<16, 1>(); run<20, 1>(); run<32, 1>(); run<40, 1>(); run<80, 1>();
  return 0;
}
"""


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope="module")
def transforms(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("regfft")
    src, exe = d / "regfft_host.cpp", d / "regfft_host"
    src.write_text(PROGRAM)
    # host code only: the transforms are __host__ __device__
    r = subprocess.run([hipcc, "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    res = {}
    for line in out.strip().splitlines():
        f = line.split()
        n, sign = int(f[0]), int(f[1])
        v = np.array([float(t) for t in f[2:]]).reshape(n, 2)
        res[(n, sign)] = v[:, 0] + 1j * v[:, 1]
    return res


@pytest.mark.parametrize("sign", (-1, 1))
@pytest.mark.parametrize("n", SIZES)
def test_register_fft_is_the_dft(transforms, n, sign):
    i = np.arange(n)
    x = (np.sin(1.3 * i + 0.2).astype(np.float32).astype(np.float64)
         + 1j * np.cos(0.7 * i * i + 0.1).astype(np.float32).astype(np.float64))
    # X[k] = sum_j x[j] exp(sign 2 pi i j k / n), written out (no FFT library)
    k = i[:, None]
    ref = (x[None, :] * np.exp(sign * 2j * np.pi * k * i[None, :] / n)).sum(axis=1)
    got = transforms[(n, sign)]
    # FP32 transforms: a few ulp of the largest output per stage
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max() * np.log2(n + 1), (n, sign)
