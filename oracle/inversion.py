"""C_l -> P_inf inversion and the closed forms tying C_l, xi and P (test infrastructure only).

Sec. II A-B of the paper:
* xi_sph(theta) = sum_l (2l+1) C_l P_l(cos theta) / 4 pi                  (eq. harmonics)
* chord between two points of a sphere of radius R at angle theta: 2 R sin(theta/2)  (eq. rtheta)
* xi_inf(r) = 4 pi int_0^inf k^2 P_inf(k) j0(k r) dk                       (eq. xiinfpinf)
* the programme min c.x s.t. A x >= b, x >= 0 with c_j = sum_i A_ij       (eq. sumconstraint)
  on constraints r_i = i dr (dr = R b / 5, up to r_max = 2 R sin(theta_max)) and unknowns
  x_j = P_inf(k_j), k_j = j dk (dk = 2 pi / (3 r_max)). The box reads the table as linear
  between nodes and zero beyond the last, P_inf = sum_j x_j phi_j with phi_j the hat of
  node j, so A_ij = 4 pi int k^2 j0(k r_i) phi_j(k) dk: the rising half of the hat on
  [k_{j-1}, k_j] and the falling half on [k_j, k_{j+1}] (none after the last node), each
  integrated by a 16-point Gauss-Legendre rule (SciPy's nodes and weights).
* C_l of the box field sampled on a full shell of radius R:
  C_l^box = 4 pi sum_{f != 0} P_box(|k_f|) j_l(|k_f| R)^2 (expand e^{i k.R n} in spherical
  harmonics and average |a_lm|^2 over m).
* the expected pseudo-C_l of maps observed on a polar cap of half-angle theta_c:
  2 pi int xi(theta) P_l(cos theta) w(theta) sin(theta) dtheta, with w the cap's pair
  weight; it depends on xi only at separations inside the cap, which is all a cap-limited
  programme constrains (for the full sphere it inverts eq. harmonics).

Everything here is written from those definitions with SciPy's Legendre, spherical Bessel
and HiGHS routines as library steps.
"""
import functools
import math

import numpy as np
import scipy.integrate
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
    A = hat_integrals(r, k)
    c = A.sum(axis=0)
    return r, b, k, A, c


def hat_integrals(r, k):
    """A[i, j] = 4 pi int k^2 j0(k r_i) phi_j(k) dk over the two halves of each hat."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    x, w = scipy.special.roots_legendre(16)
    A = np.zeros((r.size, k.size))

    def half(a, c, rising):
        t = 0.5 * (c - a) * x + 0.5 * (c + a)
        phi = (t - a) / (c - a) if rising else (c - t) / (c - a)
        f = 4.0 * math.pi * t**2 * phi * (0.5 * (c - a) * w)
        return scipy.special.spherical_jn(0, np.outer(r, t)) @ f

    for j in range(k.size):
        if j > 0:
            A[:, j] += half(k[j - 1], k[j], True)
        if j + 1 < k.size:
            A[:, j] += half(k[j], k[j + 1], False)
    return A


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


def xi_inf_of(k, p, r):
    """xi_inf(r) of a tabulated P_inf, read as linear between its nodes (eq. xiinfpinf
    through the programme's hat integrals)."""
    k = np.asarray(k, dtype=np.float64)
    return hat_integrals(r, k) @ np.asarray(p, dtype=np.float64)


def cap_pair_weight(theta, theta_cap):
    """w(theta): (1 / 4 pi) x the measure of ordered pixel pairs of a polar cap of half-angle
    theta_cap at angular separation theta, per unit solid angle of the second point's
    direction ring (w = 1 for the full sphere). For each theta, SciPy's adaptive quadrature
    integrates over the first point's colatitude a the in-cap share of the ring of radius
    theta around it, with a break at a = |theta_cap - theta| where that share stops being
    the whole ring (or nothing)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    if theta_cap >= math.pi:
        return np.ones_like(theta)
    ctc = math.cos(theta_cap)

    def share(a, t):
        sa, st = math.sin(a), math.sin(t)
        if sa * st == 0.0:
            return 1.0 if math.cos(a - t) >= ctc else 0.0
        c = (ctc - math.cos(a) * math.cos(t)) / (sa * st)
        return math.acos(min(1.0, max(-1.0, c))) / math.pi

    out = np.empty_like(theta)
    for i, t in enumerate(theta):
        val, _ = scipy.integrate.quad(lambda a: share(a, t) * math.sin(a), 0.0, theta_cap,
                                      points=[abs(theta_cap - t)], limit=200, epsabs=1e-14, epsrel=1e-12)
        out[i] = 2 * math.pi * val / (4 * math.pi)
    return out


@functools.lru_cache(maxsize=8)
def _cap_nodes(theta_cap, n_theta):
    """Separation nodes and weights w(theta) sin(theta) dtheta of the cap integral below
    (remembered per cap: the pair weight is the slow part)."""
    x, wq = np.polynomial.legendre.leggauss(n_theta)
    if theta_cap >= math.pi / 2:
        edges = [0.0, math.pi]
    else:
        edges = [0.0, theta_cap, 2 * theta_cap]
    th = np.concatenate([lo + 0.5 * (hi - lo) * (x + 1) for lo, hi in zip(edges[:-1], edges[1:])])
    wt = np.concatenate([0.5 * (hi - lo) * wq for lo, hi in zip(edges[:-1], edges[1:])])
    return th, cap_pair_weight(th, theta_cap) * np.sin(th) * wt


def cap_pseudo_cl(xi_of_theta, theta_cap, lmax, n_theta=2000):
    """Expected pseudo-C_l of maps with correlation xi(theta) observed on a polar cap:
    2 pi int xi(theta) P_l(cos theta) w(theta) sin(theta) dtheta over in-cap separations,
    Gauss-Legendre on [0, theta_cap] and [theta_cap, 2 theta_cap] (w has a kink at
    theta_cap). For the full sphere (w = 1) this inverts eq. harmonics. A list of xi
    functions gives a list of spectra (one evaluation of w)."""
    if isinstance(xi_of_theta, (list, tuple)):
        fns = xi_of_theta
    else:
        return cap_pseudo_cl([xi_of_theta], theta_cap, lmax, n_theta)[0]
    th, g = _cap_nodes(float(theta_cap), int(n_theta))
    fs = [fn(th) * g for fn in fns]
    outs = [np.empty(lmax + 1) for _ in fns]
    for l in range(lmax + 1):
        pl = scipy.special.eval_legendre(l, np.cos(th))
        for f, out in zip(fs, outs):
            out[l] = 2 * math.pi * np.sum(f * pl)
    return outs
