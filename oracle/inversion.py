"""C_l -> P_inf inversion and the closed forms tying C_l, xi and P (test infrastructure only).

Sec. II A-B of the paper:
* xi_sph(theta) = sum_l (2l+1) C_l P_l(cos theta) / 4 pi                  (eq. harmonics)
* chord between two points of a sphere of radius R at angle theta: 2 R sin(theta/2)  (eq. rtheta)
* xi_inf(r) = 4 pi int_0^inf k^2 P_inf(k) j0(k r) dk                       (eq. xiinfpinf)
* the programme min c.x s.t. A x >= b, x >= 0 with c_j = sum_i A_ij       (eq. sumconstraint)
  on constraints r_i = i dr (dr = R b / 5, up to r_max = 2 R sin(theta_max)) and unknowns
  x_j = P_inf(k_j), k_j = j dk (dk = 2 pi / (3 r_max)), A_ij = 4 pi k_j^2 j0(k_j r_i) dk.
* C_l of the box field sampled on a full shell of radius R:
  C_l^box = 4 pi sum_{f != 0} P_box(|k_f|) j_l(|k_f| R)^2 (expand e^{i k.R n} in spherical
  harmonics and average |a_lm|^2 over m).

Everything here is written from those definitions with SciPy's Legendre, spherical Bessel
and HiGHS routines as library steps.
"""
import math

import numpy as np
import scipy.optimize
import scipy.special

from . import spectrum


def xi_sph(theta, cl):
    """eq. harmonics, summed term by term with scipy's Legendre polynomials."""
    x = np.cos(np.asarray(theta, dtype=np.float64))
    out = np.zeros_like(x)
    for l, c in enumerate(np.asarray(cl, dtype=np.float64)):
        if c != 0.0:
            out += (2 * l + 1) * c * scipy.special.eval_legendre(l, x) / (4 * math.pi)
    return out


def chord(theta, R):
    """eq. rtheta for a sphere of radius R."""
    return 2.0 * R * np.sin(np.asarray(theta) / 2.0)


def programme(cl, R, theta_max, beam, k_max):
    """(r, b, k, A, c) of the discretised programme, from the definitions above."""
    r_max = 2.0 * R * math.sin(min(theta_max, math.pi / 2))
    dr = R * beam / 5.0
    n_r = int(math.floor(r_max / dr + 1e-9)) + 1
    r = np.array([i * dr for i in range(n_r)])
    theta = 2.0 * np.arcsin(np.minimum(r / (2.0 * R), 1.0))
    b = xi_sph(theta, cl)
    dk = 2.0 * math.pi / (3.0 * r_max)
    n_k = int(math.floor(k_max / dk + 1e-9)) + 1
    k = np.array([j * dk for j in range(n_k)])
    A = np.empty((n_r, n_k))
    for j in range(n_k):
        A[:, j] = 4.0 * math.pi * k[j] ** 2 * scipy.special.spherical_jn(0, k[j] * r) * dk
    c = A.sum(axis=0)
    return r, b, k, A, c


def solve(A, b, c):
    """Optimal value and a solution of min c.x, A x >= b, x >= 0 (x_0 = 0), by HiGHS'
    interior-point method with crossover, in units scaled by b_0 and the column norms."""
    col = np.where(np.abs(A).max(axis=0) > 0, np.abs(A).max(axis=0), 1.0)
    As, bs = A / col, b / b[0]
    bounds = [(0.0, 0.0)] + [(0.0, None)] * (A.shape[1] - 1)
    res = scipy.optimize.linprog(As.sum(axis=0), A_ub=-As, b_ub=-bs, bounds=bounds, method="highs-ipm")
    if res.status != 0:
        raise RuntimeError(res.message)
    x = np.maximum(res.x, 0.0) * b[0] / col
    return float(c @ x), x


def xi_inf_gaussian(r, amp, s):
    """xi_inf for P_inf = amp exp(-k^2 s^2 / 2): amp (2 pi)^{3/2} / s^3 exp(-r^2 / 2 s^2)."""
    return amp * (2 * math.pi) ** 1.5 / s**3 * np.exp(-np.asarray(r) ** 2 / (2 * s * s))


def cl_gaussian(lmax, amp, s, R):
    """C_l on a sphere of radius R of the field with xi_inf = amp exp(-r^2 / 2 s^2):
    4 pi amp e^{-x} i_l(x), x = R^2 / s^2 (modified spherical Bessel i_l)."""
    x = R * R / (s * s)
    l = np.arange(lmax + 1)
    # e^{-x} i_l(x) = sqrt(pi / 2x) I_{l+1/2}(x) e^{-x}
    return 4 * math.pi * amp * np.sqrt(math.pi / (2 * x)) * scipy.special.ive(l + 0.5, x)


def cl_box(N, L, R, k_tab, p_tab, lmax):
    """Expected full-shell C_l (l = 0..lmax) of the box field, grouped by |f|^2."""
    pb = spectrum.p_box_table(N, L, k_tab, p_tab)
    f = np.arange(N)
    f2 = np.minimum(f, N - f) ** 2
    m = (f2[:, None, None] + f2[None, :, None] + f2[None, None, :]).ravel()
    mult = np.bincount(m, minlength=pb.size)
    used = np.nonzero((mult > 0) & (pb > 0))[0]
    kk = (2 * math.pi / L) * np.sqrt(used.astype(np.float64))
    w = mult[used] * pb[used]
    out = np.empty(lmax + 1)
    for l in range(lmax + 1):
        out[l] = 4 * math.pi * np.sum(w * scipy.special.spherical_jn(l, kk * R) ** 2)
    return out
