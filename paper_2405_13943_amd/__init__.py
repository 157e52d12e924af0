"""MI355X-native (gfx950, HIP) hot path of ADMM-consensus Gaussian splatting.

The compute lives in the C-ABI library ``libgs.so`` (``include/gs.h``);
``paper_2405_13943_amd.gs`` is its thin ctypes binding.  Submodules are
imported lazily so that the input generators (``scenes``) can be used
without loading the GPU library.
"""
__all__ = ["scenes", "gs", "raster", "admm", "serve"]
