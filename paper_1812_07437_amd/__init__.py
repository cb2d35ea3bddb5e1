"""MI355X-native weak-lensing P+B covariance library (libwlcov) and its binding.

``paper_1812_07437_amd.wlcov`` is the ctypes binding of the C ABI declared in
``include/wlcov.h``; ``paper_1812_07437_amd.build`` compiles the HIP sources
for gfx950.
"""
