"""From an angular power spectrum C_l to the 3-D spectrum P_inf(k) of the box (host, FP64).

Giner Mascarell & Bunn, Sec. II A-B. The correlation on the sphere is
xi_sph(theta) = sum_l (2l+1) C_l P_l(cos theta) / (4 pi) (eq. harmonics); two points of a
sphere of radius R at angle theta are a chord r = 2 R sin(theta/2) apart (eq. rtheta); an
isotropic 3-D spectrum gives xi_inf(r) = 4 pi int k^2 P_inf(k) j0(k r) dk (eq. xiinfpinf).
Matching xi_inf to xi_sph at chords up to r_max, with P_inf >= 0, is a linear programme:
minimise c.x subject to A x >= b, x >= 0, where x_j = P_inf(k_j), b_i = xi_sph(theta_i),
A_ij = 4 pi k_j^2 j0(k_j r_i) dk and c_j = sum_i A_ij, so that c.x = sum_i (A x)_i is
smallest when every constraint holds with equality (eq. sumconstraint).

Discretisation (Sec. II B): constraints at r_i = i dr, dr = R b / 5, up to
r_max = 2 R sin(theta_max) (the widest chord of a cap of polar angle theta_max; theta_max
>= 90 deg gives the full shell, r_max = 2R); unknowns at k_j = j dk, dk = 2 pi / (3 r_max),
up to k_max (the paper does not fix it; the default is the box's isotropic band limit
pi N / L). b is the Gaussian beam width of C_l^smooth = C_l exp(-b^2 l^2) (eq. cl); for the
synthetic spectra with a damping exp(-(l/l_d)^2), b = 1/l_d.

This is setup work done once per spectrum; the result is the (k, P_inf) table passed to
cmbx_spectrum_table.
"""
import math

import numpy as np


def xi_sph(theta, cl):
    """xi_sph(theta) = sum_l (2l+1) C_l P_l(cos theta) / 4 pi, by the Legendre recurrence."""
    x = np.cos(np.asarray(theta, dtype=np.float64))
    cl = np.asarray(cl, dtype=np.float64)
    p_prev = np.ones_like(x)
    out = cl[0] * p_prev
    if cl.size > 1:
        p = x.copy()
        out = out + 3.0 * cl[1] * p
        for l in range(1, cl.size - 1):
            p_next = ((2 * l + 1) * x * p - l * p_prev) / (l + 1)
            p_prev, p = p, p_next
            out = out + (2 * (l + 1) + 1) * cl[l + 1] * p
    return out / (4.0 * math.pi)


def _j0(x):
    x = np.asarray(x, dtype=np.float64)
    safe = np.where(x == 0.0, 1.0, x)
    return np.where(x == 0.0, 1.0, np.sin(safe) / safe)


def lp_problem(cl, R, theta_max, beam, k_max):
    """The discretised programme: dict(r, theta, b, k, A, c)."""
    th = min(float(theta_max), 0.5 * math.pi)
    r_max = 2.0 * R * math.sin(th)
    dr = R * beam / 5.0
    n_r = int(math.floor(r_max / dr + 1e-9)) + 1
    r = dr * np.arange(n_r)
    theta = 2.0 * np.arcsin(np.clip(r / (2.0 * R), 0.0, 1.0))
    b = xi_sph(theta, cl)
    dk = 2.0 * math.pi / (3.0 * r_max)
    n_k = int(math.floor(k_max / dk + 1e-9)) + 1
    k = dk * np.arange(n_k)
    A = 4.0 * math.pi * (k[None, :] ** 2) * _j0(k[None, :] * r[:, None]) * dk
    c = A.sum(axis=0)
    return dict(r=r, theta=theta, b=b, k=k, A=A, c=c, dr=dr, dk=dk, r_max=r_max)


def invert(cl, R, theta_max, beam, N=None, L=1.0, k_max=None):
    """Solve the programme with HiGHS; returns (k, P_inf, info). P_inf(0) is fixed to 0
    (the k = 0 column of A is zero). Raises RuntimeError if the solver fails."""
    from scipy.optimize import linprog

    if k_max is None:
        if N is None:
            raise ValueError("give N (and L) or k_max")
        k_max = math.pi * N / L
    pr = lp_problem(cl, R, theta_max, beam, k_max)
    A, b = pr["A"], pr["b"]
    # The same programme in well-scaled units (HiGHS tolerances are absolute): constraints
    # divided by xi_sph(0) and unknowns by their column norms 4 pi k^2 dk, so that the
    # scaled unknown y_j is the fraction of xi(0) carried by node j.
    xi0 = float(b[0])
    if not xi0 > 0.0:
        raise ValueError("xi_sph(0) must be positive")
    col = 4.0 * math.pi * pr["k"] ** 2 * pr["dk"]
    col[0] = 1.0
    As = A / col[None, :]
    bs = b / xi0
    cs = As.sum(axis=0)
    bounds = [(0.0, 0.0)] + [(0.0, None)] * (A.shape[1] - 1)
    res = linprog(cs, A_ub=-As, b_ub=-bs, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(f"linear programme failed: {res.message}")
    y = np.maximum(res.x, 0.0)
    x = y * xi0 / col
    x[0] = 0.0
    fit = A @ x
    info = dict(objective=float(pr["c"] @ x), sum_b=float(b.sum()), n_r=A.shape[0], n_k=A.shape[1],
                max_rel_excess=float(((fit - b) / xi0).max()), min_rel_excess=float(((fit - b) / xi0).min()),
                xi0=xi0, xi0_fit=float(fit[0]), nonzero=int((y > 0).sum()))
    return pr["k"], x, info


def beam_from_damping(ld):
    """exp(-(l/l_d)^2) = exp(-b^2 l^2) with b = 1/l_d (eq. cl)."""
    return 1.0 / float(ld)
