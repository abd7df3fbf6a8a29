"""ctypes binding of libshwfs (include/shwfs.h): argument marshalling only.

Every step of the measurement runs in the HIP kernels of the library.
Device buffers are torch tensors on the ROCm device (torch names it
"cuda"); streams are torch streams.  There is no CPU fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libshwfs.so")

ABI_VERSION = 1
OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_ABI = 0, -1, -2, -3, -4, -5
FLAG_NOISE = 1
PRECISION_SHIFT = 4
PREC_FP32, PREC_BF16, PREC_BF16X3, PREC_FP16X3 = 0, 1, 2, 3

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libshwfs.so not built at {LIB_PATH}: run `python -m paper_1408_0698_amd.build`")
_lib = C.CDLL(LIB_PATH)


class WfsConfigC(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("pupil_n", C.c_int32), ("pupil_dx_m", C.c_double),
        ("obstruction", C.c_double), ("n_subap", C.c_int32), ("fft_n", C.c_int32), ("conv_n", C.c_int32),
        ("det_n", C.c_int32), ("lgs", C.c_int32), ("flags", C.c_uint32), ("min_illum", C.c_double),
        ("wavelength_m", C.c_double), ("na_height_m", C.c_double), ("na_fwhm_m", C.c_double),
        ("elong_max_arcsec", C.c_double), ("spot_fwhm_arcsec", C.c_double),
        ("photons_per_subap", C.c_double), ("ron_e", C.c_double), ("threshold_e", C.c_double),
    ]


class LgsGeomC(C.Structure):
    _fields_ = [("launch_x_m", C.c_double), ("launch_y_m", C.c_double)]


class WorkC(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("d_opd_m", C.c_void_p), ("row_pitch", C.c_int64),
                ("wfs_stride", C.c_int64), ("seed", C.c_uint64), ("frame", C.c_uint64),
                ("d_slopes", C.c_void_p), ("d_images", C.c_void_p)]


_P = C.c_void_p
_sig = {
    "shw_last_error": (C.c_char_p, []),
    "shw_abi_version": (C.c_int32, []),
    "shw_wfs_config_check": (C.c_int, [C.POINTER(WfsConfigC), C.c_int32, C.POINTER(LgsGeomC)]),
    "shw_wfs_geometry": (C.c_int, [C.POINTER(WfsConfigC), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double)]),
    "shw_wfs_plan_create": (C.c_int, [C.POINTER(WfsConfigC), C.c_int32, C.POINTER(LgsGeomC), C.POINTER(_P)]),
    "shw_wfs_plan_create_sodium": (C.c_int, [C.POINTER(WfsConfigC), C.c_int32, C.POINTER(LgsGeomC), C.c_int32,
                                             C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(_P)]),
    "shw_wfs_plan_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]),
    "shw_wfs_plan_kernel_spectra": (C.c_int, [_P, C.c_int32, _P, _P]),
    "sh_wfs_measure": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_uint64, C.c_uint64,
                                 _P, _P, _P, _P]),
    "sh_wfs_measure_sodium": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_uint64,
                                        C.c_uint64, _P, _P, _P, _P]),
    "sh_wfs_measure_batch": (C.c_int, [C.POINTER(WorkC), C.c_int32, _P]),
    "shw_wfs_plan_destroy": (C.c_int, [_P]),
    "shw_wfs_plan_variant_count": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "shw_wfs_plan_set_variant": (C.c_int, [_P, C.c_int32]),
    "shw_wfs_plan_get_variant": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "shw_wfs_plan_autotune": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _P, C.c_int32, _P,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "shw_wfs_plan_variant_params": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "shw_wfs_plan_set_noise_head": (C.c_int, [_P, C.c_int32]),
    "shw_wfs_plan_get_noise_head": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "shw_wfs_plan_autotune_noise_head": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _P, C.c_int32,
                                                   _P, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "sh_wfs_measure_devframe": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_uint64, _P,
                                          _P, _P, _P, _P]),
    "sh_wfs_measure_devframe_at": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_uint64, _P,
                                             C.c_uint32, _P, _P, _P, _P]),
    "shw_counter_add": (C.c_int, [_P, C.c_uint64, _P]),
    "shw_graph_begin": (C.c_int, [_P]),
    "shw_graph_end": (C.c_int, [_P, C.POINTER(_P)]),
    "shw_graph_launch": (C.c_int, [_P, _P]),
    "shw_graph_destroy": (C.c_int, [_P]),
    "shw_psf_plan_create": (C.c_int, [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double,
                                      C.POINTER(_P)]),
    "psf_accumulate": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int32, _P, _P, _P]),
    "psf_accumulate_stars": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _P, C.c_int64,
                                       _P, _P]),
    "shw_psf_plan_destroy": (C.c_int, [_P]),
    "shw_dm_plan_create": (C.c_int, [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double,
                                     C.c_double, C.c_int32, C.POINTER(_P)]),
    "shw_dm_plan_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "shw_dm_geometry": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "shw_dm_surface": (C.c_int, [_P, _P, _P, _P]),
    "shw_dm_plan_destroy": (C.c_int, [_P]),
    "shw_dm_influence_opd": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64,
                                       C.c_int64, _P]),
    "shw_push_pull": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_float, _P, C.c_int64, _P]),
    "shw_recon_plan_create": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(_P)]),
    "shw_recon_step": (C.c_int, [_P, _P, C.c_int64, _P, C.c_float, _P, _P, _P]),
    "shw_recon_plan_destroy": (C.c_int, [_P]),
    "shw_residual_opd": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _P, C.c_int64, C.c_int64, _P]),
    "shw_project_layers": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_int32,
                                     C.POINTER(C.c_double), _P, _P, C.c_int64, C.c_int64, _P]),
    "shw_uplink_tilt": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                                  C.c_double, C.c_int32, _P, _P]),
    "psf_encircled_energy": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_double), _P, _P]),
    "psf_encircled_energy_noalloc": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_double), _P,
                                                 _P]),
    "psf_resample_accumulate": (C.c_int, [C.c_int32, _P, C.c_double, C.c_float, _P, _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class ShwError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: code {code}: {last_error()}")


def last_error() -> str:
    return _lib.shw_last_error().decode()


def _check(code, where):
    if code != OK:
        raise ShwError(code, where)


def make_config(cfg) -> WfsConfigC:
    """C struct from any object with the WfsConfig attributes."""
    c = WfsConfigC()
    c.abi_version = ABI_VERSION
    for name, _ in WfsConfigC._fields_:
        if name == "abi_version":
            continue
        setattr(c, name, getattr(cfg, name))
    return c


def _geom_array(launch):
    if launch is None:
        return None, None
    arr = (LgsGeomC * len(launch))(*[LgsGeomC(float(x), float(y)) for x, y in launch])
    return arr, C.cast(arr, C.POINTER(LgsGeomC))


def config_check(cfg, n_wfs=1, launch=None) -> int:
    arr, ptr = _geom_array(launch)
    c = make_config(cfg)
    return _lib.shw_wfs_config_check(C.byref(c), n_wfs, ptr)


def geometry(cfg):
    """(valid_idx list, illum list) from the library's host code."""
    c = make_config(cfg)
    n = C.c_int32(0)
    _check(_lib.shw_wfs_geometry(C.byref(c), C.byref(n), None, None), "shw_wfs_geometry")
    idx = (C.c_int32 * max(1, n.value))()
    il = (C.c_double * max(1, n.value))()
    _check(_lib.shw_wfs_geometry(C.byref(c), C.byref(n), idx, il), "shw_wfs_geometry")
    return list(idx)[: n.value], list(il)[: n.value]


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class WfsPlan:
    """n_wfs Shack-Hartmann sensors of one geometry (plan owned by the library)."""

    def __init__(self, cfg, n_wfs=1, launch=None, sodium=None):
        """sodium: optional (dh_m, weight) sequences: the sodium sub-layer form of an LGS sensor."""
        self.cfg = cfg
        self.n_wfs = n_wfs
        self._c = make_config(cfg)
        arr, ptr = _geom_array(launch)
        h = C.c_void_p()
        self.n_sub = 0
        if sodium is None:
            _check(_lib.shw_wfs_plan_create(C.byref(self._c), n_wfs, ptr, C.byref(h)), "shw_wfs_plan_create")
        else:
            dh, wt = (list(map(float, v)) for v in sodium)
            n = len(dh)
            if len(wt) != n:
                raise ValueError("sodium heights and weights differ in length")
            _check(_lib.shw_wfs_plan_create_sodium(C.byref(self._c), n_wfs, ptr, n, (C.c_double * max(1, n))(*dh),
                                                   (C.c_double * max(1, n))(*wt), C.byref(h)),
                   "shw_wfs_plan_create_sodium")
            self.n_sub = n
        self._h = h
        nv = C.c_int32(0)
        nb = C.c_size_t(0)
        _check(_lib.shw_wfs_plan_info(self._h, C.byref(nv), C.byref(nb)), "shw_wfs_plan_info")
        self.n_valid = nv.value
        self.device_bytes = nb.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:   # the module may be torn down first
            _lib.shw_wfs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def kernel_spectra(self, wfs, out, stream=None):
        _check(_lib.shw_wfs_plan_kernel_spectra(self._h, wfs, _ptr(out), _stream_ptr(stream)),
               "shw_wfs_plan_kernel_spectra")
        return out

    @property
    def n_variants(self):
        n = C.c_int32(0)
        _check(_lib.shw_wfs_plan_variant_count(self._h, C.byref(n)), "shw_wfs_plan_variant_count")
        return n.value

    @property
    def variant(self):
        v = C.c_int32(0)
        _check(_lib.shw_wfs_plan_get_variant(self._h, C.byref(v)), "shw_wfs_plan_get_variant")
        return v.value

    def set_variant(self, v):
        _check(_lib.shw_wfs_plan_set_variant(self._h, v), "shw_wfs_plan_set_variant")

    VARIANT_PARAM_NAMES = ("convolution", "waves_per_eu", "persistent", "noise_kernel", "items_per_block",
                           "sublayers")
    CONVOLUTION_FORMS = ("whole_rows", "split_rows", "band_limited")

    def variant_params(self, v):
        """The parameters launch variant v fixes, as a dict."""
        out = (C.c_int32 * 6)()
        _check(_lib.shw_wfs_plan_variant_params(self._h, v, out), "shw_wfs_plan_variant_params")
        d = dict(zip(self.VARIANT_PARAM_NAMES, list(out)))
        d["convolution"] = self.CONVOLUTION_FORMS[d["convolution"]]
        return d

    @property
    def noise_head(self):
        h = C.c_int32(0)
        _check(_lib.shw_wfs_plan_get_noise_head(self._h, C.byref(h)), "shw_wfs_plan_get_noise_head")
        return h.value

    def set_noise_head(self, head):
        _check(_lib.shw_wfs_plan_set_noise_head(self._h, head), "shw_wfs_plan_set_noise_head")

    def autotune_noise_head(self, opd, slopes, reps=20, stream=None):
        """Time the noise kernel's inversion head (2, 4, 6 steps) for the current variant; keep the
        fastest.  Returns (best, [ms per launch for 2, 4, 6])."""
        ms = (C.c_float * 3)()
        best = C.c_int32(-1)
        _check(_lib.shw_wfs_plan_autotune_noise_head(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0),
                                                     opd.shape[0], _ptr(slopes), reps, _stream_ptr(stream),
                                                     C.byref(best), ms), "shw_wfs_plan_autotune_noise_head")
        return best.value, list(ms)

    def autotune(self, opd, slopes, reps=20, stream=None):
        """Time every launch variant on these inputs; select the fastest (the plan's default when it is
        within 2 % of the fastest).  Returns (best, [ms per launch])."""
        n = self.n_variants
        ms = (C.c_float * n)()
        best = C.c_int32(-1)
        _check(_lib.shw_wfs_plan_autotune(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0),
                                          opd.shape[0], _ptr(slopes), reps, _stream_ptr(stream), C.byref(best), ms),
               "shw_wfs_plan_autotune")
        return best.value, list(ms)

    def measure_devframe(self, opd, slopes, d_frame0, images=None, flags=None, seed=0, stream=None, frame_offset=0):
        """As measure, with the first frame number read on the device from the uint64 tensor d_frame0
        (plus frame_offset)."""
        if opd.dim() != 4 or opd.stride(3) != 1:
            raise ValueError("opd must be [frames][wfs][rows][cols] with contiguous rows")
        if frame_offset == 0:
            _check(_lib.sh_wfs_measure_devframe(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0),
                                                opd.shape[0], seed, _ptr(d_frame0), _ptr(slopes), _ptr(images),
                                                _ptr(flags), _stream_ptr(stream)), "sh_wfs_measure_devframe")
        else:
            _check(_lib.sh_wfs_measure_devframe_at(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0),
                                                   opd.shape[0], seed, _ptr(d_frame0), frame_offset, _ptr(slopes),
                                                   _ptr(images), _ptr(flags), _stream_ptr(stream)),
                   "sh_wfs_measure_devframe_at")
        return slopes

    def measure(self, opd, slopes, images=None, flags=None, seed=0, frame0=0, stream=None):
        """opd: float32 device tensor [F][W][N][N] (last dim contiguous); slopes [F][W][2][n_valid]."""
        if opd.dim() != 4 or opd.stride(3) != 1:
            raise ValueError("opd must be [frames][wfs][rows][cols] with contiguous rows")
        nf = opd.shape[0]
        _check(_lib.sh_wfs_measure(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0), nf,
                                   seed, frame0, _ptr(slopes), _ptr(images), _ptr(flags),
                                   _stream_ptr(stream)), "sh_wfs_measure")
        return slopes


    def measure_sodium(self, opd, slopes, images=None, flags=None, seed=0, frame0=0, stream=None):
        """opd: float32 device tensor [F][W][n_sub][N][N] (a sub-layer stride of 0 shares one wavefront)."""
        if opd.dim() != 5 or opd.stride(4) != 1:
            raise ValueError("opd must be [frames][wfs][sub-layers][rows][cols] with contiguous rows")
        _check(_lib.sh_wfs_measure_sodium(self._h, _ptr(opd), opd.stride(3), opd.stride(2), opd.stride(1),
                                          opd.stride(0), opd.shape[0], seed, frame0, _ptr(slopes), _ptr(images),
                                          _ptr(flags), _stream_ptr(stream)), "sh_wfs_measure_sodium")
        return slopes


def measure_batch(items, stream=None):
    """items: list of (plan, opd[W][N][N], slopes[W][2][S], images or None, seed, frame)."""
    arr = (WorkC * max(1, len(items)))()
    for k, (plan, opd, slopes, images, seed, frame) in enumerate(items):
        arr[k] = WorkC(plan.handle.value, opd.data_ptr(), opd.stride(1), opd.stride(0), seed, frame,
                       slopes.data_ptr(), images.data_ptr() if images is not None else None)
    _check(_lib.sh_wfs_measure_batch(arr, len(items), _stream_ptr(stream)), "sh_wfs_measure_batch")


class PsfPlan:
    """Science PSF accumulation over frames (Strehl per frame)."""

    def __init__(self, pupil_n, pupil_dx_m, obstruction, fft_m, wavelength_m):
        h = C.c_void_p()
        _check(_lib.shw_psf_plan_create(ABI_VERSION, pupil_n, pupil_dx_m, obstruction, fft_m, wavelength_m,
                                        C.byref(h)), "shw_psf_plan_create")
        self._h = h
        self.fft_m = fft_m
        self.pupil_n = pupil_n
        self.wavelength_m = wavelength_m

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:   # the module may be torn down first
            _lib.shw_psf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def accumulate(self, opd, acc, strehl=None, stream=None):
        """opd: float32 device tensor [F][N][N] (rows contiguous); acc [M][M] (+=); strehl [F] or None."""
        if opd.dim() != 3 or opd.stride(2) != 1:
            raise ValueError("opd must be [frames][rows][cols] with contiguous rows")
        _check(_lib.psf_accumulate(self._h, _ptr(opd), opd.stride(1), opd.stride(0), opd.shape[0], _ptr(acc),
                                   _ptr(strehl), _stream_ptr(stream)), "psf_accumulate")
        return acc

    def accumulate_stars(self, opd, acc, strehl=None, stream=None):
        """opd: float32 device [S][F][N][N] (rows contiguous); acc [S][M][M] (+=); strehl [S][F] or None."""
        if opd.dim() != 4 or opd.stride(3) != 1:
            raise ValueError("opd must be [stars][frames][rows][cols] with contiguous rows")
        _check(_lib.psf_accumulate_stars(self._h, _ptr(opd), opd.stride(2), opd.stride(1), opd.stride(0), opd.shape[1],
                                         opd.shape[0], _ptr(acc), acc.stride(0), _ptr(strehl), _stream_ptr(stream)),
               "psf_accumulate_stars")
        return acc


    def encircled_energy(self, psf, radii_px, out=None, stream=None, noalloc=False):
        """psf: float32 device [M][M] or [S][M][M]; radii in pixels -> float64 device [S][n_r] (or [n_r]).
        noalloc: call psf_encircled_energy_noalloc (static device workspace, no allocation; out must
        then be given)."""
        import torch
        single = psf.dim() == 2
        p3 = psf.unsqueeze(0) if single else psf
        if p3.dim() != 3 or p3.shape[1:] != (self.fft_m, self.fft_m) or p3.stride(2) != 1 or p3.stride(1) != self.fft_m:
            raise ValueError("psf must be [S][M][M] with contiguous rows of the plan's size")
        r = (C.c_double * len(radii_px))(*[float(v) for v in radii_px])
        if noalloc and out is None:
            raise ValueError("noalloc needs an output tensor")
        if out is None:
            out = torch.empty((p3.shape[0], len(radii_px)), dtype=torch.float64, device=psf.device)
        if (out.dtype != torch.float64 or not out.is_contiguous() or out.dim() != 2
                or tuple(out.shape) != (p3.shape[0], len(radii_px))):
            raise ValueError("out must be a contiguous float64 [S][n_r] tensor")
        fn = _lib.psf_encircled_energy_noalloc if noalloc else _lib.psf_encircled_energy
        _check(fn(self._h, _ptr(p3), p3.shape[0], p3.stride(0), len(radii_px), r, _ptr(out), _stream_ptr(stream)),
               "psf_encircled_energy_noalloc" if noalloc else "psf_encircled_energy")
        return out[0] if single else out


def psf_resample_accumulate(src, scale, weight, dst, stream=None):
    """dst[M][M] += weight * src (a PSF at wavelength lambda_i) on the grid of lambda_ref, scale = lambda_ref / lambda_i."""
    m = src.shape[-1]
    if src.shape != (m, m) or dst.shape != (m, m) or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("src and dst must be contiguous [M][M]")
    _check(_lib.psf_resample_accumulate(m, _ptr(src), float(scale), float(weight), _ptr(dst), _stream_ptr(stream)),
           "psf_resample_accumulate")
    return dst


def polychromatic_psf(plans, weights, opd, out, strehl=None, stream=None):
    """Colour-weighted PSF on the angular grid of plans[0]'s wavelength (Sec. 3 PSF block).

    plans: PsfPlan per wavelength (same pupil and M); weights: the object's colour, one per plan;
    opd: float32 device [F][N][N]; out [M][M] += sum_i w_i sum_f P_i,f resampled to plans[0]'s grid.
    strehl: optional float32 device [len(plans)][F] of per-wavelength Strehl ratios.  Device work
    runs in the library (accumulation per wavelength, then psf_resample_accumulate).
    """
    import torch
    m = plans[0].fft_m
    tmp = torch.empty((m, m), dtype=torch.float32, device=out.device)
    for i, (p, w) in enumerate(zip(plans, weights)):
        if p.fft_m != m:
            raise ValueError("all plans must have the same M")
        tmp.zero_()
        p.accumulate(opd, tmp, None if strehl is None else strehl[i], stream=stream)
        psf_resample_accumulate(tmp, plans[0].wavelength_m / p.wavelength_m, w, out, stream=stream)
    return out


def _layer_args(layers):
    """layers: sequence of (screen float32 device [R][C] with unit column stride, spacing_m, altitude_m, x0, y0)."""
    n = len(layers)
    ptrs = (C.c_void_p * n)(*[_ptr(l[0]) for l in layers])
    rows = (C.c_int32 * n)(*[l[0].shape[0] for l in layers])
    cols = (C.c_int32 * n)(*[l[0].shape[1] for l in layers])
    pitch = (C.c_int64 * n)(*[l[0].stride(0) for l in layers])
    for l in layers:
        if l[0].dim() != 2 or l[0].stride(1) != 1:
            raise ValueError("screens must be [rows][cols] with unit column stride")
    par = (C.c_double * (4 * n))(*[float(v) for l in layers for v in l[1:5]])
    return n, ptrs, rows, cols, pitch, par


def project_layers(layers, pupil_n, dx_m, targets, out, tilt=None, stream=None):
    """Cone-effect open-loop wavefronts: targets = [(theta_x, theta_y, altitude_m or 0)], out float32 [T][N][N]."""
    n, ptrs, rows, cols, pitch, par = _layer_args(layers)
    tp = (C.c_double * (3 * max(1, len(targets))))(*[float(v) for t in targets for v in t])
    if out.dim() != 3 or out.stride(2) != 1:
        raise ValueError("out must be [targets][rows][cols] with contiguous rows")
    _check(_lib.shw_project_layers(n, ptrs, rows, cols, pitch, par, pupil_n, dx_m, len(targets), tp, _ptr(tilt),
                                   _ptr(out), out.stride(1), out.stride(0), _stream_ptr(stream)), "shw_project_layers")
    return out


def uplink_tilt(layers, lgs, llt_diameter_m, n_samples, out, stream=None):
    """lgs = [(launch_x_m, launch_y_m, theta_x, theta_y, sodium_altitude_m)]; out float64 device [n][2] radians."""
    n, ptrs, rows, cols, pitch, par = _layer_args(layers)
    lp = (C.c_double * (5 * max(1, len(lgs))))(*[float(v) for g in lgs for v in g])
    _check(_lib.shw_uplink_tilt(n, ptrs, rows, cols, pitch, par, len(lgs), lp, llt_diameter_m, n_samples, _ptr(out),
                                _stream_ptr(stream)), "shw_uplink_tilt")
    return out


def dm_geometry(pupil_n, pupil_dx_m, alt_m, pitch_px, field_radius_arcsec):
    """(actuator positions [n][2] as a list of (x, y) px, surface side) from the library's host code."""
    n = C.c_int32(0)
    size = C.c_int32(0)
    _check(_lib.shw_dm_geometry(pupil_n, pupil_dx_m, alt_m, pitch_px, field_radius_arcsec, C.byref(n),
                                C.byref(size), None), "shw_dm_geometry")
    xy = (C.c_double * (2 * max(1, n.value)))()
    _check(_lib.shw_dm_geometry(pupil_n, pupil_dx_m, alt_m, pitch_px, field_radius_arcsec, C.byref(n),
                                C.byref(size), xy), "shw_dm_geometry")
    v = list(xy)[: 2 * n.value]
    return [(v[2 * k], v[2 * k + 1]) for k in range(n.value)], size.value


class DmPlan:
    """One deformable mirror: actuator grid and influence functions (plan owned by the library)."""

    def __init__(self, pupil_n, pupil_dx_m, alt_m, pitch_px, field_radius_arcsec, coupling=0.3, patch=64):
        h = C.c_void_p()
        _check(_lib.shw_dm_plan_create(ABI_VERSION, pupil_n, pupil_dx_m, alt_m, pitch_px, field_radius_arcsec,
                                       coupling, patch, C.byref(h)), "shw_dm_plan_create")
        self._h = h
        n = C.c_int32(0)
        size = C.c_int32(0)
        _check(_lib.shw_dm_plan_info(self._h, C.byref(n), C.byref(size), None), "shw_dm_plan_info")
        self.n_act = n.value
        self.size = size.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:   # the module may be torn down first
            _lib.shw_dm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def influence_opd(self, act, amp, row0, col0, pupil_n, out, stream=None):
        """out[k] = amp[k] * IF of actuator act[k] on the pupil window (row0, col0); act int32, amp float32."""
        _check(_lib.shw_dm_influence_opd(self._h, _ptr(act), _ptr(amp), act.shape[0], row0, col0, pupil_n, _ptr(out),
                                         out.stride(-2), out.stride(0), _stream_ptr(stream)), "shw_dm_influence_opd")
        return out

    def surface(self, coefs, out, stream=None):
        """coefs: float32 device [n_act]; out: float32 device [size][size] (contiguous)."""
        _check(_lib.shw_dm_surface(self._h, _ptr(coefs), _ptr(out), _stream_ptr(stream)), "shw_dm_surface")
        return out


def residual_opd(screen, surfaces, pupil_n, scr_origin, dm_origin, out, stream=None):
    """out[k] = screen window k - sum_d surface_d window (k, d).

    screen: float32 device [R][Cols] (rows contiguous); surfaces: list of square contiguous float32 device
    arrays; scr_origin: [n_out][2] ints; dm_origin: [n_out][n_dm][2] ints; out: float32 device [n_out][N][N].
    """
    n_out = len(scr_origin)
    n_dm = len(surfaces)
    ptrs = (C.c_void_p * max(1, n_dm))(*[s.data_ptr() for s in surfaces])
    sizes = (C.c_int32 * max(1, n_dm))(*[s.shape[0] for s in surfaces])
    so = (C.c_int32 * (2 * max(1, n_out)))(*[int(v) for o in scr_origin for v in o])
    do = (C.c_int32 * (2 * max(1, n_out * n_dm)))(*[int(v) for o in dm_origin for dd in o for v in dd])
    _check(_lib.shw_residual_opd(_ptr(screen), screen.shape[0], screen.shape[1], screen.stride(0), n_dm, ptrs, sizes,
                                 pupil_n, n_out, so, do, _ptr(out), out.stride(1), out.stride(0),
                                 _stream_ptr(stream)), "shw_residual_opd")
    return out


class ReconPlan:
    """Control-matrix product and pure integrator of the closed loop."""

    def __init__(self, n_modes, n_slopes):
        h = C.c_void_p()
        _check(_lib.shw_recon_plan_create(n_modes, n_slopes, C.byref(h)), "shw_recon_plan_create")
        self._h = h
        self.n_modes = n_modes
        self.n_slopes = n_slopes

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:   # the module may be torn down first
            _lib.shw_recon_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, cm, slopes, gain, coefs, delta=None, stream=None):
        """coefs += gain * cm @ slopes; cm float32 device [n_modes][ld] (rows contiguous), slopes [n_slopes]."""
        _check(_lib.shw_recon_step(self._h, _ptr(cm), cm.stride(0), _ptr(slopes), gain, _ptr(coefs), _ptr(delta),
                                   _stream_ptr(stream)), "shw_recon_step")
        return coefs


def counter_add(d_counter, inc=1, stream=None):
    """d_counter (uint64 device tensor, one element) += inc, as a kernel on the stream."""
    _check(_lib.shw_counter_add(_ptr(d_counter), inc, _stream_ptr(stream)), "shw_counter_add")


class Graph:
    """A captured loop step: library calls issued on `stream` inside `with Graph.capture(stream)`."""

    def __init__(self, handle):
        self._h = handle

    @staticmethod
    def capture(stream):
        return _Capture(stream)

    def launch(self, stream=None):
        _check(_lib.shw_graph_launch(self._h, _stream_ptr(stream)), "shw_graph_launch")

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:   # the module may be torn down first
            _lib.shw_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class _Capture:
    def __init__(self, stream):
        self.stream = stream
        self.graph = None

    def __enter__(self):
        _check(_lib.shw_graph_begin(_stream_ptr(self.stream)), "shw_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = C.c_void_p()
        rc = _lib.shw_graph_end(_stream_ptr(self.stream), C.byref(h))
        if exc_type is None:
            _check(rc, "shw_graph_end")
            self.graph = Graph(h)
        elif rc == OK:
            _lib.shw_graph_destroy(h)
        return False


def push_pull(slopes, n_modes, scale, im, stream=None):
    """im[s, m] (row pitch im.stride(0)) = (slopes[2m] - slopes[2m+1])[s] * scale; slopes [2 n_modes][n_slopes]."""
    _check(_lib.shw_push_pull(_ptr(slopes), n_modes, slopes.shape[-1], scale, _ptr(im), im.stride(0),
                              _stream_ptr(stream)), "shw_push_pull")
    return im
