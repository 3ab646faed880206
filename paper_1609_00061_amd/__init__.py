"""MI355X-native pixel array method (arXiv 1609.00061): plotting of polynomial
relations as bit-packed Boolean arrays and Boolean generalized array
multiplication, as hand-written HIP kernels for gfx950 behind a C ABI.

Importing the package is cheap; the compiled library is loaded on first use
of `paper_1609_00061_amd.pa` (see `pa.load()`).
"""
__all__ = ["inputs", "pa"]
