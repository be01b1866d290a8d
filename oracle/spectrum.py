"""Box power spectrum and per-mode weight tables (test infrastructure only).

Sec. II C of the paper: replacing the Fourier integral of the infinite-space spectrum by a
sum over the box's wave vectors gives P_box = P_inf dk_x dk_y dk_z (eq. pboxandinf), with
dk = 2 pi / (N dp) along the N-point sides and 2 pi / (M dp) along the M-point side
(eqs. smalldeltakxy, smalldeltakz), i.e. P_box = P_inf (2 pi / dp)^3 / (M N^2)
(eq. finalpbox). For the cubic box used here (M = N, N dp = L) that is
P_box = P_inf (2 pi / L)^3.

A box mode with integer frequency vector (f_x, f_y, f_z) has |k| = (2 pi / L) sqrt(m),
m = f_x^2 + f_y^2 + f_z^2, so every weight the simulator needs is indexed by the integer
m in [0, 3 (N/2)^2]. The table of the user's P_inf(k) is interpolated linearly in k and
taken as zero outside its range (the paper's k_max beyond which P = 0, Sec. II B). The
k = 0 mode carries no power.

Weights (FP64, rounded once to the working precision by the caller):
  half[m] = sqrt(P_box(k_m) / 2)   for a generic mode, whose real and imaginary parts
                                    each carry half the variance;
  full[m] = sqrt(P_box(k_m))       for the self-conjugate modes, which are real.
"""
import numpy as np

TWO_PI = 6.283185307179586  # 2 pi rounded to binary64


def interp_p(k_tab, p_tab, k):
    """P_inf at wave numbers ``k``: piecewise linear in k, zero outside [k_tab[0], k_tab[-1]]."""
    k_tab = np.asarray(k_tab, dtype=np.float64)
    p_tab = np.asarray(p_tab, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    n = k_tab.size
    i = np.searchsorted(k_tab, k, side="right") - 1
    i = np.clip(i, 0, n - 2)
    d = k - k_tab[i]
    h = k_tab[i + 1] - k_tab[i]
    t = d / h
    p = p_tab[i] + (p_tab[i + 1] - p_tab[i]) * t
    inside = (k >= k_tab[0]) & (k <= k_tab[-1])
    return np.where(inside, p, 0.0)


def lattice_k(N, L):
    """|k| for m = 0 .. 3 (N/2)^2: (2 pi / L) sqrt(m)."""
    c = TWO_PI / L
    m = np.arange(3 * (N // 2) ** 2 + 1, dtype=np.float64)
    return c * np.sqrt(m)


def p_box_table(N, L, k_tab, p_tab):
    """P_box(k_m) for every integer m = |f|^2, with P_box(0) = 0."""
    c = TWO_PI / L
    c3 = c * c * c
    p = interp_p(k_tab, p_tab, lattice_k(N, L)) * c3
    p[0] = 0.0
    return p


def weight_tables(N, L, k_tab, p_tab):
    """(half, full): sqrt(P_box / 2) and sqrt(P_box) per integer m, in FP64."""
    p = p_box_table(N, L, k_tab, p_tab)
    half = np.sqrt(p * 0.5)
    full = np.sqrt(p)
    return half, full


def mode_m(N, ix=None):
    """Integer |f|^2 for every half-grid mode, shape (N, N, N/2 + 1), or (len(ix), N, N/2 + 1)
    for the x-indices ``ix`` only."""
    f = np.arange(N)
    f = np.minimum(f, N - f)
    fx = f if ix is None else f[np.asarray(ix)]
    fz = np.arange(N // 2 + 1)
    return (fx[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2).astype(np.int64)


def lattice_xi0(N, L, k_tab, p_tab):
    """Sum of P_box over the full N^3 lattice: the variance <T^2> of the box field (eq. pboxxi at r = 0)."""
    p = p_box_table(N, L, k_tab, p_tab)
    f = np.arange(N)
    f = np.minimum(f, N - f)
    m = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    return float(p[m].sum())
