"""MI355X-native CG-FFT discrete dipole approximation.

The compute path is ``libdda.so`` (hand-written HIP kernels for gfx950 behind a
C ABI, declared in ``include/dda.h``); ``paper_0908_0863_amd.dda`` is the thin
ctypes binding.  Importing this package loads nothing: the library is opened on
first use and its absence raises.
"""
__all__ = ["dda", "inputs"]
