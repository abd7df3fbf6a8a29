"""MI355X-native Shack-Hartmann wavefront-sensor measurement and science PSF.

The compute path is libshwfs (HIP kernels for gfx950 behind the C ABI of
include/shwfs.h); ``shwfs`` is its Python binding.  Importing ``shwfs``
fails loudly when the library has not been built.
"""
__all__ = ["shwfs", "build"]
