"""C-ABI tests that need no GPU: the library loads, exports every declared
symbol, validates arguments on the host, and its host geometry agrees
with the oracle's independently computed tables."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from gen import configs as G
from oracle import geometry as OG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1408_0698_amd import shwfs
    return shwfs


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "shwfs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([a-z_][a-z0-9_]*)\s*\(", txt, re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("sh_wfs_measure", "psf_accumulate", "shw_wfs_plan_create", "shw_last_error",
                 "sh_wfs_measure_batch", "shw_psf_plan_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(os.path.join(ROOT, "paper_1408_0698_amd", "lib", "libshwfs.so"))
    for name in _declared_functions():
        assert hasattr(lib, name), name
    s = _lib()
    assert set(_declared_functions()) == set(s.EXPORTED)
    assert s._lib.shw_abi_version() == s.ABI_VERSION


@pytest.mark.parametrize("cfg,n_wfs", [(G.CFG0, 1), (G.CFG1, 6), (G.CFG1_R2, 6)])
def test_supported_workloads_pass_validation(cfg, n_wfs):
    s = _lib()
    launch = G.launch_positions(cfg, n_wfs) if cfg.lgs else None
    assert s.config_check(cfg, n_wfs, launch) == s.OK, s.last_error()


@pytest.mark.parametrize("change,code", [
    (dict(pupil_n=81), -1),                 # n_subap does not divide pupil_n
    (dict(fft_n=12), -4),                   # not a multiple of the sub-aperture size: no kernel
    (dict(fft_n=4), -1),                    # smaller than the sub-aperture
    (dict(conv_n=17), -1),                  # odd padding
    (dict(det_n=0), -1),
    (dict(det_n=17), -1),                   # larger than conv_n
    (dict(obstruction=1.0), -1),
    (dict(wavelength_m=0.0), -1),
    (dict(wavelength_m=float("nan")), -1),
    (dict(min_illum=0.0), -1),
    (dict(photons_per_subap=-1.0), -1),
    (dict(flags=1 << 12), -1),              # unknown flag bit
    (dict(fft_n=24, conv_n=24), -4),        # valid geometry, no kernel compiled
])
def test_invalid_configs_are_rejected_on_host(change, code):
    s = _lib()
    cfg = G.CFG0.replace(**change)
    assert s.config_check(cfg, 1, None) == code
    assert s.last_error() != ""


def test_abi_version_and_nulls():
    s = _lib()
    c = s.make_config(G.CFG0)
    c.abi_version = 99
    assert s._lib.shw_wfs_config_check(C.byref(c), 1, None) == s.E_ABI
    assert s._lib.shw_wfs_config_check(None, 1, None) == s.E_INVALID
    assert s.config_check(G.CFG0, 0, None) == s.E_INVALID
    assert s.config_check(G.CFG1, 6, None) == s.E_INVALID  # LGS needs launch positions
    out = C.c_void_p()
    assert s._lib.shw_wfs_plan_create(None, 1, None, C.byref(out)) == s.E_INVALID
    assert s._lib.sh_wfs_measure(None, None, 0, 0, 0, 1, 0, 0, None, None, None, None) == s.E_INVALID
    assert s._lib.psf_accumulate(None, None, 0, 0, 1, None, None, None) == s.E_INVALID
    assert s._lib.sh_wfs_measure_batch(None, 1, None) == s.E_INVALID
    assert s._lib.sh_wfs_measure_batch(None, 0, None) == s.OK
    assert s._lib.shw_psf_plan_create(s.ABI_VERSION, 800, 0.05, 0.14, 1000, 1.65e-6, C.byref(out)) == s.E_UNSUPPORTED
    assert s._lib.shw_psf_plan_create(s.ABI_VERSION, 800, 0.05, 0.14, 400, 1.65e-6, C.byref(out)) == s.E_INVALID
    assert s._lib.shw_psf_plan_create(2, 800, 0.05, 0.14, 1600, 1.65e-6, C.byref(out)) == s.E_ABI
    assert s._lib.shw_wfs_plan_destroy(None) == s.OK


@pytest.mark.parametrize("cfg", [G.CFG0, G.CFG1, G.CFG4_NGS, G.CFG0.replace(obstruction=0.3, min_illum=0.75)])
def test_host_geometry_matches_oracle(cfg):
    s = _lib()
    idx, il = s.geometry(cfg)
    vi, oil = OG.subap_table(cfg)
    assert idx == list(vi)
    assert np.array_equal(np.array(il), oil)


@pytest.mark.parametrize("alt,pitch,n_want,size_want", [(0.0, 10, 5025, 800), (4000.0, 20, 1413, 848),
                                                         (12700.0, 20, 1781, 952)])
def test_host_dm_geometry_matches_oracle(alt, pitch, n_want, size_want):
    from oracle import dm as OD
    s = _lib()
    act, size = s.dm_geometry(800, 4.875e-2, alt, pitch, 60.0)
    want = OD.actuators(800, 4.875e-2, alt, pitch, 60.0)
    assert len(act) == n_want == len(want) and size == size_want
    assert np.array_equal(np.array(act), want)
    assert size == OD.surface_size(800, 4.875e-2, alt, 60.0)


def test_dm_and_residual_argument_checks():
    s = _lib()
    out = C.c_void_p()
    assert s._lib.shw_dm_plan_create(s.ABI_VERSION, 801, 0.05, 0.0, 10, 60.0, 0.3, 64, C.byref(out)) == s.E_INVALID
    assert s._lib.shw_dm_plan_create(s.ABI_VERSION, 800, 0.05, 0.0, 10, 60.0, 1.3, 64, C.byref(out)) == s.E_INVALID
    assert s._lib.shw_dm_plan_create(s.ABI_VERSION, 800, 0.05, 0.0, 10, 60.0, 0.3, 63, C.byref(out)) == s.E_INVALID
    assert s._lib.shw_dm_plan_create(s.ABI_VERSION, 800, 0.05, 0.0, 0, 60.0, 0.3, 64, C.byref(out)) == s.E_INVALID
    assert s._lib.shw_dm_surface(None, None, None, None) == s.E_INVALID
    so = (C.c_int32 * 2)(10, 1300)   # window leaves a 2048-wide screen
    fake = C.c_void_p(16)
    assert s._lib.shw_residual_opd(fake, 2048, 2048, 2048, 0, None, None, 800, 1, so, None, fake, 800, 640000,
                                   None) == s.E_INVALID
    assert s._lib.shw_residual_opd(fake, 2048, 2048, 2048, 5, None, None, 800, 1, so, None, fake, 800, 640000,
                                   None) == s.E_INVALID
    assert s._lib.shw_residual_opd(fake, 2048, 2048, 2048, 0, None, None, 800, 0, so, None, fake, 800, 640000,
                                   None) == s.OK


def test_calibration_argument_checks():
    """shw_dm_influence_opd and shw_push_pull reject bad windows and layouts before any launch."""
    import ctypes as C

    from paper_1408_0698_amd import shwfs as s
    fake = C.c_void_p(0x1000)
    assert s._lib.shw_dm_influence_opd(None, fake, fake, 1, 0, 0, 8, fake, 8, 64, None) == s.E_INVALID
    assert s._lib.shw_push_pull(fake, 4, 10, C.c_float(1.0), fake, 3, None) == s.E_INVALID
    assert s._lib.shw_push_pull(None, 4, 10, C.c_float(1.0), fake, 4, None) == s.E_INVALID
    assert s._lib.shw_push_pull(fake, -1, 10, C.c_float(1.0), fake, 4, None) == s.E_INVALID
    assert s._lib.shw_push_pull(fake, 0, 10, C.c_float(1.0), None, 4, None) == 0


def test_sodium_plan_argument_checks():
    """Sub-layer plans are validated on the host before any HIP call."""
    import ctypes as C

    from gen import configs as G
    from paper_1408_0698_amd import shwfs as s
    h = C.c_void_p()
    launch = G.launch_positions(G.CFG1, 1)
    geom = (s.LgsGeomC * 1)(s.LgsGeomC(*launch[0]))
    dh = (C.c_double * 3)(-1000.0, 0.0, 1000.0)
    wt = (C.c_double * 3)(1.0, 2.0, 1.0)
    cfg = s.make_config(G.CFG1)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 0, dh, wt, C.byref(h)) == s.E_INVALID
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 17, dh, wt, C.byref(h)) == s.E_INVALID
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 3, None, wt, C.byref(h)) == s.E_INVALID
    bad = (C.c_double * 3)(1.0, -2.0, 1.0)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 3, dh, bad, C.byref(h)) == s.E_INVALID
    zero = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 3, dh, zero, C.byref(h)) == s.E_INVALID
    low = (C.c_double * 3)(-1e6, 0.0, 1000.0)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(cfg), 1, geom, 3, low, wt, C.byref(h)) == s.E_INVALID
    ngs = s.make_config(G.CFG0)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(ngs), 1, geom, 3, dh, wt, C.byref(h)) == s.E_INVALID
    mfma = s.make_config(G.CFG1.replace(flags=G.PREC_FP16X3 << 4))
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(mfma), 1, geom, 3, dh, wt, C.byref(h)) == s.E_UNSUPPORTED
    r2 = s.make_config(G.CFG1_R2)
    assert s._lib.shw_wfs_plan_create_sodium(C.byref(r2), 1, geom, 3, dh, wt, C.byref(h)) == s.E_UNSUPPORTED
    assert s._lib.sh_wfs_measure_sodium(None, None, 800, 0, 0, 0, 1, 0, 0, None, None, None, None) == s.E_INVALID


def test_geometry_and_psf_extras_argument_checks():
    """Layer projection, uplink tilt, encircled energy and resampling validate on the host."""
    s = _lib()
    fake = C.c_void_p(0x1000)
    ptrs = (C.c_void_p * 2)(0x1000, 0x2000)
    rows = (C.c_int32 * 2)(400, 400)
    cols = (C.c_int32 * 2)(400, 400)
    pitch = (C.c_int64 * 2)(400, 400)
    # (spacing, altitude, x0, y0): a ground layer and one at 8 km, axis at the screen centre
    par = (C.c_double * 8)(0.1, 0.0, 200.0, 200.0, 0.1, 8000.0, 200.0, 200.0)
    tgt = (C.c_double * 3)(0.0, 0.0, 90000.0)
    args = (2, ptrs, rows, cols, pitch, par)
    # a 20 m pupil (200 samples of 0.1 m) fits; 50 m leaves the 40 m screens
    ok_call = s._lib.shw_project_layers(*args, 200, 0.1, 0, tgt, None, fake, 200, 40000, None)
    assert ok_call == s.OK   # no targets: nothing to do
    assert s._lib.shw_project_layers(*args, 500, 0.1, 1, tgt, None, fake, 500, 250000, None) == s.E_INVALID
    low = (C.c_double * 3)(0.0, 0.0, 5000.0)   # source below the 8 km layer
    assert s._lib.shw_project_layers(*args, 200, 0.1, 1, low, None, fake, 200, 40000, None) == s.E_INVALID
    tilted = (C.c_double * 3)(2e-3, 0.0, 0.0)  # 8 km x 2 mrad = 16 m: the footprint leaves the screen
    assert s._lib.shw_project_layers(*args, 200, 0.1, 1, tilted, None, fake, 200, 40000, None) == s.E_INVALID
    assert s._lib.shw_project_layers(*args, 200, 0.1, 2, (C.c_double * 6)(*[0.0] * 6), None, fake, 200, 100,
                                     None) == s.E_INVALID   # outputs overlap
    bad = (C.c_double * 8)(0.0, 0.0, 200.0, 200.0, 0.1, 8000.0, 200.0, 200.0)
    assert s._lib.shw_project_layers(2, ptrs, rows, cols, pitch, bad, 200, 0.1, 1, tgt, None, fake, 200, 40000,
                                     None) == s.E_INVALID
    assert s._lib.shw_project_layers(17, ptrs, rows, cols, pitch, par, 200, 0.1, 1, tgt, None, fake, 200, 40000,
                                     None) == s.E_INVALID
    lgs = (C.c_double * 5)(19.0, 0.0, 0.0, 0.0, 90000.0)
    far = (C.c_double * 5)(25.0, 0.0, 0.0, 0.0, 90000.0)  # launcher 25 m off axis: beam leaves the 20 m half-width
    assert s._lib.shw_uplink_tilt(*args, 1, far, 0.4, 32, fake, None) == s.E_INVALID
    assert s._lib.shw_uplink_tilt(*args, 1, lgs, 0.0, 32, fake, None) == s.E_INVALID
    assert s._lib.shw_uplink_tilt(*args, 1, lgs, 0.4, 1, fake, None) == s.E_INVALID
    assert s._lib.shw_uplink_tilt(*args, 0, lgs, 0.4, 32, None, None) == s.OK
    assert s._lib.psf_encircled_energy(None, fake, 1, 0, 1, (C.c_double * 1)(3.0), fake, None) == s.E_INVALID
    assert s._lib.psf_encircled_energy_noalloc(None, fake, 1, 0, 1, (C.c_double * 1)(3.0), fake, None) == s.E_INVALID
    assert s._lib.shw_wfs_plan_set_noise_head(None, 4) == s.E_INVALID
    assert s._lib.shw_wfs_plan_variant_params(None, 0, (C.c_int32 * 6)()) == s.E_INVALID
    assert s._lib.psf_resample_accumulate(1, fake, 1.0, C.c_float(1.0), C.c_void_p(0x9000), None) == s.E_INVALID
    assert s._lib.psf_resample_accumulate(64, fake, 0.0, C.c_float(1.0), C.c_void_p(0x90000), None) == s.E_INVALID
    assert s._lib.psf_resample_accumulate(64, fake, 1.0, C.c_float(1.0), C.c_void_p(0x1100), None) == s.E_INVALID


def test_issue_probe_library_is_separate_and_checks_arguments():
    """The VALU issue probe (bench.py --valu-probe) is its own library, not part of the boundary:
    it exports its two entry points, libshwfs does not, and bad sizes are refused on the host."""
    probe = C.CDLL(os.path.join(ROOT, "paper_1408_0698_amd", "lib", "libshw_probe.so"))
    probe.shw_probe_valu.restype = C.c_int
    probe.shw_probe_valu.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    probe.shw_probe_valu_kinds.restype = C.c_int
    assert probe.shw_probe_valu_kinds() == 6
    buf = (C.c_float * 256)()
    assert probe.shw_probe_valu(0, 0, 16, C.cast(buf, C.c_void_p), None) == -1      # no blocks
    assert probe.shw_probe_valu(0, 1, 0, C.cast(buf, C.c_void_p), None) == -1      # no iterations
    assert probe.shw_probe_valu(0, 1, 16, None, None) == -1                       # no output
    assert probe.shw_probe_valu(6, 1, 16, C.cast(buf, C.c_void_p), None) == -1    # no such kind
    lib = C.CDLL(os.path.join(ROOT, "paper_1408_0698_amd", "lib", "libshwfs.so"))
    assert not hasattr(lib, "shw_probe_valu")
