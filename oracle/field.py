"""Inverse 3-D DFT of the half grid to the real box field (test infrastructure only).

Sec. II D 1: the simulated map is the inverse Fourier transform of the filled box. The
definition used here is the unnormalised transform with the + sign,

    T(j) = sum over all N^3 modes f of T(f) exp(+2 pi i f.j / N),   j in [0, N)^3,

where the modes outside the stored half grid are the conjugates T(-f) = conj T(f). The
result is real. The sum is evaluated with SciPy's pocketfft inverse real transform in
FP64 (``norm="forward"`` leaves the inverse unscaled); the brute-force sum above pins it
in the tests.
"""
import numpy as np
import scipy.fft


def field(h, workers=None):
    """Real field (N, N, N), float64, from a half grid (N, N, N/2 + 1)."""
    h = np.asarray(h)
    N = h.shape[0]
    if h.shape != (N, N, N // 2 + 1):
        raise ValueError("half grid must have shape (N, N, N/2 + 1)")
    return scipy.fft.irfftn(h.astype(np.complex128), s=(N, N, N), axes=(0, 1, 2),
                            norm="forward", workers=workers)
