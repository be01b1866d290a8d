"""Flat N x N x M boxes: the 3-D Fourier method on them and the 2-D (hybrid) Fourier
method (test infrastructure only).

Sec. II C: the box has N points along x and y and M along z, spaced dp in every
direction; its wave numbers are spaced 2 pi / (N dp) along x, y and 2 pi / (M dp) along z
(eqs. smalldeltakxy, smalldeltakz), so P_box = P_inf (2 pi / dp)^3 / (M N^2) (eq.
finalpbox). A mode with integer frequencies (f_x, f_y, f_z) has
|k| = (2 pi / dp) sqrt((f_x^2 + f_y^2) / N^2 + f_z^2 / M^2). P_box depends on the mode
through s = f_x^2 + f_y^2 and |f_z| only, so the tables here are indexed [s][|f_z|].

Layout of every field here: layers [z][x][y] (y fastest); node (ix, iy, iz) at
(ix dp, iy dp, iz dp), periodic in x and y with period N dp.

3-D Fourier method on the flat box (Sec. II D 1): every mode of the N x N x M lattice is a
complex normal of variance P_box; the real field is made from the half grid in y
(iy = 0 .. N/2, all ix, all iz): generic modes half[s][|fz|] (g_re + i g_im) with
half = sqrt(P_box / 2); on the planes iy = 0 and N/2 the mode (ix, iz) and its partner
(-ix mod N, -iz mod M) are conjugate, the one with the smaller ix M + iz drawn; the
self-conjugate modes (ix in {0, N/2}, iz in {0, M/2} on those planes) are real,
sqrt(P_box) g_re. Normal pair of mode (ix, iy, iz): Philox counter (iz >> 1, iy, ix, 2)
through the canonical Box-Muller (``normal``). Field: the unnormalised inverse DFT with
the + sign over the whole lattice.

2-D Fourier method (Sec. II D 2): only h consecutive layers z_j = j dp (j < h) of the same
N x N x M box are made, in the hybrid space T^(k_x, k_y, z). For each column (k_x, k_y)
the values at different heights are correlated with
Gamma_jk = xi_{k_x k_y}(z_j - z_k), xi_{k_x k_y}(z) = sum over f_z of P_box e^{i k_z z}:
P_box filled into the N x N x M lattice and transformed along z. A column is drawn as
S (g_re + i g_im) / sqrt 2 with independent unit normals g (S g_re for the four
self-conjugate columns, which are real), where S S^T = Gamma. The paper factors Gamma by
its eigendecomposition P D P^T (eq. gammasvd, its adopted choice) and applies P D^{1/2};
here the factor is the symmetric square root P D^{1/2} P^T of the same decomposition
(eigenvalues below zero, from rounding, set to zero): P^T g is again a vector of
independent unit normals, so the maps have the same statistics, and unlike P D^{1/2} the
symmetric root is unique, so two implementations agree. The rows iy = 0 and N/2 are
Hermitian in k_x (the column (ix, iy) and (-ix mod N, iy) conjugate, the smaller ix
drawn). Normals of column (ix, iy), layer j: Philox counter (j >> 1, iy, ix, 1), words
(x0, x1) for even j and (x2, x3) for odd j. Layers: the inverse 2-D DFT over (k_x, k_y).

Sampling (Sec. II D 1): pixel n at o + r n, grid position p = (r n + o) (1 / dp) per
axis in FP64 with 1 / dp formed once; the stencil of the interpolant wraps in x and y;
in z it wraps modulo M on the whole flat box, and on the h layers of the 2-D method a
pixel whose stencil leaves [0, h) is NaN (the layers are a window, not a period).
"""
import numpy as np
import scipy.fft

from . import gather as _gather
from . import normal, philox
from .spectrum import TWO_PI, interp_p

STREAM_HYBRID = 1
STREAM_FLAT = 2


# ------------------------------------------------------------------ spectrum
def s_max(N):
    return 2 * (N // 2) ** 2


def p_box_flat(N, M, dp, k_tab, p_tab):
    """P_box[s][fz] for s = 0 .. 2 (N/2)^2 and fz = 0 .. M/2 (eq. finalpbox), FP64, with
    P_box(0) = 0. Operation order: q = (s M^2 + fz^2 N^2) / (N^2 M^2) (one correctly
    rounded quotient of exact integers), k = (2 pi / dp) sqrt(q),
    P_box = P_inf(k) x ((c c) c) / (M N^2), c = 2 pi / dp."""
    s = np.arange(s_max(N) + 1, dtype=np.int64)[:, None]
    fz = np.arange(M // 2 + 1, dtype=np.int64)[None, :]
    num = (s * M * M + fz * fz * N * N).astype(np.float64)
    q = num / float(N * N * M * M)
    c = TWO_PI / dp
    k = c * np.sqrt(q)
    c3 = (c * c) * c / float(M * N * N)
    p = interp_p(k_tab, p_tab, k) * c3
    p[0, 0] = 0.0
    return p


def flat_weights(N, M, dp, k_tab, p_tab):
    """(half, full) = (sqrt(P_box / 2), sqrt(P_box)) as [s][fz], FP64."""
    p = p_box_flat(N, M, dp, k_tab, p_tab)
    return np.sqrt(p * 0.5), np.sqrt(p)


def _freq(i, n):
    return np.minimum(i, n - i)


# ------------------------------------------------------------------ 3-D method, flat box
def flat_halfgrid(N, M, dp, seed, k_tab, p_tab, dtype=np.float64):
    """Modes T(ix, iy, iz) of the half grid in y, complex (N, N/2 + 1, M)."""
    rdt = np.dtype(dtype)
    cdt = np.complex128 if rdt == np.float64 else np.complex64
    half, full = flat_weights(N, M, dp, k_tab, p_tab)
    half, full = half.astype(rdt), full.astype(rdt)
    ix, iy, iz = np.meshgrid(np.arange(N), np.arange(N // 2 + 1), np.arange(M), indexing="ij")
    s = _freq(ix, N) ** 2 + _freq(iy, N) ** 2
    fz = _freq(iz, M)
    on_plane = (iy == 0) | (iy == N // 2)
    px, pz = (-ix) % N, (-iz) % M
    own, par = ix * M + iz, px * M + pz
    selfc = on_plane & (own == par)
    flip = on_plane & (own > par)
    dx, dz = np.where(flip, px, ix), np.where(flip, pz, iz)   # the mode whose words are drawn
    a, b = philox.mode_words(seed, dx, iy, dz, stream=STREAM_FLAT)
    g_re, g_im = normal.box_muller_f32(a, b) if rdt == np.float32 else normal.box_muller(a, b)
    w = np.where(selfc, full[s, fz], half[s, fz])
    zero = rdt.type(0)
    re = np.where(w == 0, zero, w * g_re)
    im = np.where(w == 0, zero, np.where(selfc, zero, w * g_im))
    out = np.empty((N, N // 2 + 1, M), dtype=cdt)
    out.real = re
    out.imag = np.where(flip, -im, im)
    return out


def flat_layers(h):
    """Real field [z][x][y] (M, N, N) of a flat half grid (N, N/2 + 1, M)."""
    N, _, M = h.shape
    # c2c along x (axis 0) and z (axis 2), c2r along y (axis 1): f[x][y][z]
    f = scipy.fft.irfftn(h.astype(np.complex128), s=(N, M, N), axes=(0, 2, 1), norm="forward")
    return np.ascontiguousarray(np.transpose(f, (2, 0, 1)))


def flat_full_grid(h):
    """Extend the half grid in y (N, N/2 + 1, M) to the whole lattice (N, N, M) by
    T(-f) = conj T(f)."""
    N, _, M = h.shape
    full = np.empty((N, N, M), dtype=h.dtype)
    full[:, : N // 2 + 1, :] = h
    ix, iz = (-np.arange(N)) % N, (-np.arange(M)) % M
    for iy in range(N // 2 + 1, N):
        full[:, iy, :] = np.conj(h[ix][:, N - iy, :][:, iz])
    return full


# ------------------------------------------------------------------ 2-D (hybrid) method
def column_xi(N, M, dp, k_tab, p_tab, h):
    """xi_s(j dp) for j = 0 .. h - 1 and every s, (s_max + 1, h): P_box over the M values of
    f_z (f_z and -f_z alike), transformed along z (unnormalised, + sign)."""
    pb = p_box_flat(N, M, dp, k_tab, p_tab)
    line = np.concatenate([pb, pb[:, 1:M - M // 2][:, ::-1]], axis=1)   # f_z = 0 .. M/2, then -(M/2 - 1) .. -1
    xi = np.fft.ifft(line, axis=1) * M
    return np.ascontiguousarray(xi.real[:, :h])


def gamma(xi_row):
    """Gamma_jk = xi(|j - k| dp) for one column."""
    h = xi_row.size
    j = np.arange(h)
    return xi_row[np.abs(j[:, None] - j[None, :])]


def sym_sqrt(G):
    """Symmetric square root P D^{1/2} P^T of symmetric matrices (..., h, h) from their
    eigendecomposition, eigenvalues below zero set to zero."""
    w, V = np.linalg.eigh(G)
    return (V * np.sqrt(np.maximum(w, 0.0))[..., None, :]) @ np.swapaxes(V, -1, -2)


def hybrid_factors(N, M, h, dp, k_tab, p_tab):
    """Symmetric roots S_s (s_max + 1, h, h) of every column's Gamma (s not a sum of two
    squares included: unused)."""
    xi = column_xi(N, M, dp, k_tab, p_tab, h)
    j = np.arange(h)
    G = xi[:, np.abs(j[:, None] - j[None, :])]
    return sym_sqrt(G)


def hybrid_columns(N, M, h, dp, seed, k_tab, p_tab, dtype=np.float64):
    """T^(ix, iy, z_j), complex (h, N, N/2 + 1): the correlated columns of the 2-D method.
    With dtype float32 the normals come from the binary32 Box-Muller (as a single-precision
    plan draws them); the factor and the products stay FP64."""
    rdt = np.dtype(dtype)
    S = hybrid_factors(N, M, h, dp, k_tab, p_tab)
    ix, iy = np.meshgrid(np.arange(N), np.arange(N // 2 + 1), indexing="ij")
    on_row = (iy == 0) | (iy == N // 2)
    px = (-ix) % N
    selfc = on_row & (ix == px)
    flip = on_row & (ix > px)
    dx = np.where(flip, px, ix)
    j = np.arange(h)
    a, b = philox.mode_words(seed, dx[None], iy[None], j[:, None, None], stream=STREAM_HYBRID)
    g_re, g_im = normal.box_muller_f32(a, b) if rdt == np.float32 else normal.box_muller(a, b)
    g_re, g_im = g_re.astype(np.float64), g_im.astype(np.float64)
    s = _freq(ix, N) ** 2 + _freq(iy, N) ** 2
    Sc = S[s]                                           # (N, N/2 + 1, h, h)
    gr = np.moveaxis(g_re, 0, -1)[..., None]            # (N, N/2 + 1, h, 1)
    gi = np.moveaxis(g_im, 0, -1)[..., None]
    vr = (Sc @ gr)[..., 0]
    vi = (Sc @ gi)[..., 0]
    inv_sqrt2 = 1.0 / np.sqrt(2.0)
    re = np.where(selfc[..., None], vr, vr * inv_sqrt2)
    im = np.where(selfc[..., None], 0.0, vi * inv_sqrt2)
    im = np.where(flip[..., None], -im, im)
    return np.moveaxis(re + 1j * im, -1, 0)


def hybrid_layers(cols):
    """Real layers [z][x][y] (h, N, N) from hybrid columns (h, N, N/2 + 1)."""
    N = cols.shape[1]
    return scipy.fft.irfftn(cols, s=(N, N), axes=(1, 2), norm="forward")


# ------------------------------------------------------------------ sampling
def positions(dp, r, dirs, observer):
    """Grid positions (n_pix, 3), FP64: p = (r n + o) (1 / dp), 1 / dp formed once."""
    dirs = np.asarray(dirs, dtype=np.float64)
    o = np.asarray(observer, dtype=np.float64).reshape(3)
    return (r * dirs + o) * (1.0 / dp)


def gather_layers(layers, dp, r, dirs, interp, observer, periodic_z):
    """Interpolated values of layers [z][x][y] at the pixels, FP64 (NaN where a stencil
    leaves a non-periodic z range)."""
    layers = np.asarray(layers, dtype=np.float64)
    nz, N, _ = layers.shape
    p = positions(dp, r, dirs, observer)
    i0 = np.floor(p)
    f = p - i0
    if interp == _gather.TRILINEAR:
        offs, kern = np.arange(0, 2), _gather.linear_kernel
    elif interp == _gather.TRICUBIC:
        offs, kern = np.arange(-1, 3), _gather.keys_kernel
    else:
        raise ValueError(interp)
    idx = i0[:, :, None].astype(np.int64) + offs[None, None, :]
    w = kern(offs[None, None, :] - f[:, :, None])
    ix, iy, iz = idx[:, 0, :] % N, idx[:, 1, :] % N, idx[:, 2, :]
    if periodic_z:
        bad = np.zeros(p.shape[0], dtype=bool)
        iz = iz % nz
    else:
        bad = (iz.min(axis=1) < 0) | (iz.max(axis=1) >= nz)
        iz = np.clip(iz, 0, nz - 1)
    K = offs.size
    out = np.zeros(p.shape[0])
    for a in range(K):
        for b in range(K):
            for c in range(K):
                out += w[:, 0, a] * w[:, 1, b] * w[:, 2, c] * layers[iz[:, c], ix[:, a], iy[:, b]]
    out[bad] = np.nan
    return out


def default_observer(N, nz, dp):
    """The centre of the layers: (N dp / 2, N dp / 2, (nz - 1) dp / 2)."""
    return np.array([0.5 * N * dp, 0.5 * N * dp, 0.5 * (nz - 1) * dp])


def observer_for_cap(N, nz, dp, r, z_min):
    """Sec. II D 2 (Fig. 2b): the middle of the simulated layers at the middle height of
    the cap about +z of radius r with edge z_min, on the axis through the layers' centre."""
    o = default_observer(N, nz, dp)
    o[2] -= r * (1.0 + z_min) / 2.0
    return o


def box_size(b, theta_max, size_factor=1.0, R=1.0):
    """The paper's box sizing (Sec. II C): dp = 0.85 dr with dr = R b / 5 (the programme's
    constraint spacing, Sec. II B); N = size_factor x the next power of two of twice the
    cap's width 2 R sin(theta_max) in points; M likewise from twice its height
    R (1 - cos theta_max). Returns (N, M, dp)."""
    dp = 0.85 * R * b / 5.0
    width = 2.0 * R * np.sin(min(theta_max, np.pi / 2)) / dp
    height = R * (1.0 - np.cos(theta_max)) / dp
    N = int(round(size_factor * (1 << int(np.ceil(np.log2(2.0 * width))))))
    M = int(round(size_factor * (1 << int(np.ceil(np.log2(2.0 * height))))))
    return N, M, dp
