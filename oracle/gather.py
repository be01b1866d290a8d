"""Sampling the box field on the sphere (test infrastructure only).

Sec. II D 1: the box map is interpolated and evaluated at the positions of the sky
pixels. Geometry: grid node j sits at j L / N (periodic), the observer at the box centre
c = (L/2, L/2, L/2), and the pixel with unit direction n at c + r n. In grid units its
position is

    p = (r n + L/2) (N / L),

evaluated in FP64 in exactly that order (r n, then + L/2, then x N/L with N/L formed
once); i0 = floor(p) and the fraction f = p - i0 then pick the stencil. Node indices wrap
modulo N.

The paper does not name the interpolant. Two are provided, both tensor products of a 1-D
kernel K evaluated at the node-to-sample distances:

* trilinear: K(x) = 1 - |x| on |x| < 1 (2 nodes per axis);
* tricubic:  Keys' cubic convolution kernel with a = -1/2 (R. Keys, IEEE Trans. ASSP 29
  (1981) 1153): K(x) = 3/2|x|^3 - 5/2|x|^2 + 1 on |x| <= 1,
  -1/2|x|^3 + 5/2|x|^2 - 4|x| + 2 on 1 < |x| < 2 (4 nodes per axis).
"""
import numpy as np

TRILINEAR = "trilinear"
TRICUBIC = "tricubic"


def keys_kernel(x):
    """Keys cubic convolution kernel, a = -1/2."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    inner = 1.5 * x**3 - 2.5 * x**2 + 1.0
    outer = -0.5 * x**3 + 2.5 * x**2 - 4.0 * x + 2.0
    return np.where(x <= 1.0, inner, np.where(x < 2.0, outer, 0.0))


def linear_kernel(x):
    x = np.abs(np.asarray(x, dtype=np.float64))
    return np.where(x < 1.0, 1.0 - x, 0.0)


def positions(N, L, r, dirs, observer=None):
    """Grid-unit positions p (n_pix, 3) of the pixels, FP64, in the fixed operation order:
    p = (r n + o) (N / L), o the observer's position in the box (default the centre, L/2
    on each axis). Sec. II D 1 places the box about the cap instead, centred on the cap's
    axis at (1 + z_min)/2 of the radius: the observer then sits below the box centre."""
    dirs = np.asarray(dirs, dtype=np.float64)
    s = N / L
    o = np.full(3, 0.5 * L) if observer is None else np.asarray(observer, dtype=np.float64).reshape(3)
    return (r * dirs + o) * s


def stencil(N, L, r, dirs, interp, observer=None):
    """Node indices (n_pix, 3, K) and 1-D weights (n_pix, 3, K) of every pixel's stencil."""
    p = positions(N, L, r, dirs, observer)
    i0 = np.floor(p)
    f = p - i0
    if interp == TRILINEAR:
        offs, kern = np.arange(0, 2), linear_kernel
    elif interp == TRICUBIC:
        offs, kern = np.arange(-1, 3), keys_kernel
    else:
        raise ValueError(interp)
    idx = (i0[:, :, None].astype(np.int64) + offs[None, None, :]) % N
    w = kern(offs[None, None, :] - f[:, :, None])
    return idx, w


def gather(fld, L, r, dirs, interp, observer=None, threads=None, chunk=1 << 16):
    """Interpolated field values at the pixels, FP64, shape (n_pix,). threads > 1 evaluates
    chunks of ``chunk`` pixels in that many threads (each pixel's sum is the same)."""
    fld = np.asarray(fld, dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float64)
    if threads is not None and threads > 1 and dirs.shape[0] > chunk:
        from concurrent.futures import ThreadPoolExecutor
        starts = range(0, dirs.shape[0], chunk)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            parts = ex.map(lambda i: gather(fld, L, r, dirs[i:i + chunk], interp, observer), starts)
            return np.concatenate(list(parts))
    N = fld.shape[0]
    idx, w = stencil(N, L, r, dirs, interp, observer)
    K = idx.shape[2]
    out = np.zeros(idx.shape[0])
    for a in range(K):
        for b in range(K):
            for c in range(K):
                out += (w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                        * fld[idx[:, 0, a], idx[:, 1, b], idx[:, 2, c]])
    return out
