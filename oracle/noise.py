"""Weighted complex Gaussian modes on the Hermitian half grid (test infrastructure only).

Sec. II D 1 of the paper fills every box mode with a complex normal of mean zero and
variance P(k) and inverse-transforms; the real part of the result is one realisation. Here
the field is made real by construction: only the half grid f_z = 0 .. N/2 is stored, and
modes obey T(-f) = conj T(f). The mode with frequency f then has E|T|^2 = P_box(|f|), so
the field's covariance is exactly sum_f P_box e^{i k.r} (eq. pboxxi).

Layout: array index i along an axis is frequency i for i <= N/2 and i - N above (for the
z axis only 0 .. N/2 are stored). Mode (ix, iy, iz) is driven by the normal pair of the
canonical stream (``philox.mode_words`` then ``normal.box_muller``):

* generic mode:            T = half[m] (g_re + i g_im)
* planes iz = 0 and N/2:   the mode and its partner (-ix mod N, -iy mod N) form a
                           conjugate pair; the one with the smaller ix N + iy is drawn as
                           above and the other is its complex conjugate;
* self-conjugate modes     (ix, iy in {0, N/2} on those planes): T = full[m] g_re, real.
* a mode whose weight is zero (P_box = 0, e.g. beyond the spectrum's k_max) is exactly
  +0 (before the conjugation of the planes' partners), whatever its normal pair.

In single precision the normal pair comes from the binary32 transform
(``normal.box_muller_f32``), the weight is rounded to FP32 and the product is an FP32
multiply; in double precision everything is binary64. Either way the result is
reproducible bit for bit.
"""
import numpy as np

from . import normal, philox, spectrum


def _pair(a, b, rdt):
    return normal.box_muller_f32(a, b) if rdt == np.float32 else normal.box_muller(a, b)


def unit_normals(N, seed, ix, dtype=np.float64):
    """(g_re, g_im) for x-index array ``ix`` (1-D) and all iy, iz; shape (len(ix), N, N/2 + 1)."""
    ix = np.asarray(ix)
    gx, gy, gz = np.meshgrid(ix, np.arange(N), np.arange(N // 2 + 1), indexing="ij")
    a, b = philox.mode_words(seed, gx, gy, gz)
    return _pair(a, b, np.dtype(dtype))


def _normals_chunk(args):
    N, seed, x0, x1, rdt = args
    return unit_normals(N, seed, np.arange(x0, x1), rdt)


def halfgrid(N, L, seed, k_tab, p_tab, dtype=np.float64, chunk=32, workers=None, threads=None):
    """The weighted half grid, complex array of shape (N, N, N/2 + 1), complex128 or complex64.
    workers > 1 draws the normals of independent x-chunks in that many processes; threads > 1
    in that many threads of this process instead (NumPy's array loops release the GIL), for
    callers that must not fork, such as a process that already drives a GPU."""
    if N % 2:
        raise ValueError("N must be even")
    rdt = np.dtype(dtype)
    cdt = np.complex128 if rdt == np.float64 else np.complex64
    half, full = spectrum.weight_tables(N, L, k_tab, p_tab)
    half = half.astype(rdt)
    full = full.astype(rdt)
    out = np.empty((N, N, N // 2 + 1), dtype=cdt)
    jobs = [(N, seed, x0, min(N, x0 + chunk), rdt) for x0 in range(0, N, chunk)]
    if threads is not None and threads > 1 and len(jobs) > 1:
        from concurrent.futures import ThreadPoolExecutor
        ex = ThreadPoolExecutor(max_workers=threads)
        normals = ex.map(_normals_chunk, jobs)
    elif workers is not None and workers > 1 and len(jobs) > 1:
        from concurrent.futures import ProcessPoolExecutor
        ex = ProcessPoolExecutor(max_workers=workers)
        normals = ex.map(_normals_chunk, jobs)
    else:
        ex, normals = None, map(_normals_chunk, jobs)
    try:
        for (_, _, x0, x1, _), (g_re, g_im) in zip(jobs, normals):
            w = half[spectrum.mode_m(N, np.arange(x0, x1))]
            zero = rdt.type(0)
            out[x0:x1].real = np.where(w == 0, zero, w * g_re)
            out[x0:x1].imag = np.where(w == 0, zero, w * g_im)
    finally:
        if ex is not None:
            ex.shutdown()
    _hermitian_planes(out, N, seed, full, rdt)
    return out


def _hermitian_planes(out, N, seed, full, rdt):
    """Impose T(-f) = conj T(f) on the planes iz = 0 and iz = N/2."""
    ix, iy = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    px, py = (-ix) % N, (-iy) % N
    own = ix * N + iy
    partner = px * N + py
    for iz in (0, N // 2):
        plane = out[:, :, iz].copy()
        mirrored = np.conj(plane[px, py])
        new = np.where(own < partner, plane, mirrored)
        selfc = own == partner
        sx, sy = ix[selfc], iy[selfc]
        a, b = philox.mode_words(seed, sx, sy, np.full(sx.shape, iz))
        g_re, _ = _pair(a, b, rdt)
        m = (np.minimum(sx, N - sx) ** 2 + np.minimum(sy, N - sy) ** 2 + iz * iz).astype(np.int64)
        new[selfc] = np.where(full[m] == 0, rdt.type(0), full[m] * g_re)
        out[:, :, iz] = new


def full_grid(h):
    """Extend a Hermitian half grid (N, N, N/2 + 1) to the full (N, N, N) spectrum."""
    N = h.shape[0]
    full = np.empty((N, N, N), dtype=h.dtype)
    full[:, :, : N // 2 + 1] = h
    ix = (-np.arange(N)) % N
    for iz in range(N // 2 + 1, N):
        full[:, :, iz] = np.conj(h[ix][:, ix][:, :, N - iz])
    return full
