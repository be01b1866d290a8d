"""MI355X-native partial-sky CMB box simulator (Giner Mascarell & Bunn, arXiv:2507.15703).

The hot path -- weighted complex Gaussian noise on the Hermitian half grid, the inverse
3-D FFT and the interpolation of the field on a sky patch -- runs in hand-written HIP
kernels for gfx950 behind the C ABI declared in ``include/cmbx.h``. ``cmbx`` is the thin
Python binding to that library; importing this package loads nothing native.
"""
