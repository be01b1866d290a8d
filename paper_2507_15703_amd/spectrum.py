"""From an angular power spectrum C_l to the 3-D spectrum P_inf(k) of the box (host, FP64).

Giner Mascarell & Bunn, Sec. II A-B. The correlation on the sphere is
xi_sph(theta) = sum_l (2l+1) C_l P_l(cos theta) / (4 pi) (eq. harmonics); two points of a
sphere of radius R at angle theta are a chord r = 2 R sin(theta/2) apart (eq. rtheta); an
isotropic 3-D spectrum gives xi_inf(r) = 4 pi int k^2 P_inf(k) j0(k r) dk (eq. xiinfpinf).
Matching xi_inf to xi_sph at chords up to r_max, with P_inf >= 0, is a linear programme:
minimise c.x subject to A x >= b, x >= 0, where x_j = P_inf(k_j), b_i = xi_sph(theta_i)
and c_j = sum_i A_ij, so that c.x = sum_i (A x)_i is smallest when every constraint holds
with equality (eq. sumconstraint).

The box reads the table as piecewise linear in k (zero beyond its last node), so A is the
integral of eq. xiinfpinf for that reading: P_inf = sum_j x_j phi_j with phi_j the hat
function of node j (1 at k_j, linear to 0 at its neighbours; the last node's hat ends at
k_j), A_ij = 4 pi int k^2 j0(k r_i) phi_j(k) dk, by Gauss-Legendre on each interval
between nodes. Then A x is exactly the correlation of the spectrum the box samples; the
plain node sum 4 pi k_j^2 j0(k_j r_i) dk is not (for the programme's sparse solutions it
put the box's xi(0) 4 % high and its correlations at half the cap's width 30 % low).

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


_GL_X, _GL_W = np.polynomial.legendre.leggauss(12)


def hat_kernel(r, k, chunk=256):
    """A[i, j] = 4 pi int k^2 j0(k r_i) phi_j(k) dk for the hat functions phi_j of the
    uniform nodes k (last node's hat ending at it), so that xi_inf(r_i) = sum_j A_ij P_j for
    the piecewise-linear P_inf through the nodes (eq. xiinfpinf). Twelve Gauss-Legendre
    points on each interval between nodes: over one interval k r changes by at most
    dk r_max = 2 pi / 3, where that rule is exact to rounding."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    k = np.asarray(k, dtype=np.float64)
    lo, hi = k[:-1], k[1:]
    h = hi - lo
    t = 0.5 * (lo + hi)[:, None] + 0.5 * h[:, None] * _GL_X[None, :]  # (intervals, 12)
    f = 4.0 * math.pi * t * t * (0.5 * h[:, None] * _GL_W[None, :])
    rise = (t - lo[:, None]) / h[:, None]  # hat of the interval's right node; 1 - rise: left node
    A = np.zeros((r.size, k.size))
    for i0 in range(0, r.size, chunk):
        J = _j0(r[i0:i0 + chunk, None, None] * t[None, :, :])
        A[i0:i0 + chunk, 1:] += np.einsum("rim,im->ri", J, f * rise)
        A[i0:i0 + chunk, :-1] += np.einsum("rim,im->ri", J, f * (1.0 - rise))
    return A


def hat_masses(k):
    """4 pi int k^2 phi_j(k) dk: the share of xi(0) that P_inf = 1 at node j alone carries."""
    return hat_kernel(np.zeros(1), k)[0]


def xi_of_table(r, k, p):
    """xi_inf at separations r of the piecewise-linear P_inf through the table (k, p)."""
    return hat_kernel(r, k) @ np.asarray(p, dtype=np.float64)


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
    A = hat_kernel(r, k)
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
    # divided by xi_sph(0) and unknowns by their hat masses (row r = 0 of A), so that the
    # scaled unknown y_j is the fraction of xi(0) carried by node j.
    xi0 = float(b[0])
    if not xi0 > 0.0:
        raise ValueError("xi_sph(0) must be positive")
    col = A[0].copy()
    col[0] = 1.0
    As = A / col[None, :]
    bs = b / xi0
    cs = As.sum(axis=0)
    bounds = [(0.0, 0.0)] + [(0.0, None)] * (A.shape[1] - 1)
    # HiGHS' default choice first; on a numerical failure its dual simplex, then its
    # interior-point method (infeasible or unbounded programmes fail in every method)
    for method in ("highs", "highs-ds", "highs-ipm"):
        res = linprog(cs, A_ub=-As, b_ub=-bs, bounds=bounds, method=method)
        if res.status == 0 or res.status in (2, 3):
            break
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


def spectrum_from_cl(cl, b, theta_max, N, L, r):
    """(k, P_inf) for the target C_l: the programme (invert) with beam b, a cap of polar
    angle theta_max (radians) on the shell of radius r, unknowns up to the band limit of an
    N^3 box of side L (pi N / L)."""
    k, p, _ = invert(cl, r, theta_max, b, N=N, L=L)
    return k, p


def synthetic_job_spectrum(N, L, r, theta_max_deg, amp=1.0):
    """(k, P_inf) of an ensemble job: the programme's solution for the synthetic C_l family
    (l_max = floor(0.8 pi r N / L), l_d = 0.6 l_max, beam 1 / l_d) scaled by ``amp``, on a
    cap of half-angle theta_max_deg, up to the box's band limit pi N / L."""
    from . import workloads
    lmax = workloads.lmax_for(N, L, r)
    cl = amp * workloads.synthetic_cl(lmax)
    k, p, _ = invert(cl, r, math.radians(theta_max_deg), 1.0 / (0.6 * lmax), N=N, L=L)
    return k, p


def beam_from_damping(ld):
    """exp(-(l/l_d)^2) = exp(-b^2 l^2) with b = 1/l_d (eq. cl)."""
    return 1.0 / float(ld)


class CapPseudoCl:
    """Expected pseudo-C_l (l = 0..lmax) of maps seen on a polar cap of half-angle theta_c.

    A map with correlation xi(theta) observed on the cap has
    E[pseudo-C_l] = 2 pi int_0^{2 theta_c} xi(theta) P_l(cos theta) w(theta) sin(theta) dtheta,
    where w(theta) is the share of ordered pixel pairs at separation theta with both ends in
    the cap (per unit solid angle of the ring around the first point, w = 1 on the full sky).
    It depends on xi only at separations the cap contains, so it compares a cap-limited
    inversion (Sec. II B) with its target C_l on equal terms.

    The theta integral is Gauss-Legendre on the panels [0, theta_c] and [theta_c, 2 theta_c]
    (w is not smooth at theta_c). w(theta) integrates, over the first point's colatitude a
    (weight sin a), the in-cap share of the ring of radius theta around it: the whole ring
    for a <= theta_c - theta, none of it for a < theta - theta_c, and between
    a0 = |theta_c - theta| and theta_c an arc whose length has a square-root edge at a0,
    removed by the substitution a = a0 + (theta_c - a0) s^2 before Gauss-Legendre in s.
    The result is a (lmax+1) x n_theta matrix acting on xi at the nodes, so each check is
    one small matrix product.
    """

    def __init__(self, theta_c, lmax, n_theta=768, n_a=192):
        self.theta_c, self.lmax = float(theta_c), int(lmax)
        u, wu = np.polynomial.legendre.leggauss(n_theta // 2)
        edges = [0.0, self.theta_c, min(math.pi, 2.0 * self.theta_c)]
        th, wt = [], []
        for lo, hi in zip(edges[:-1], edges[1:]):
            th.append(lo + 0.5 * (hi - lo) * (u + 1.0))
            wt.append(0.5 * (hi - lo) * wu)
        self.theta = np.concatenate(th)
        wt = np.concatenate(wt)
        n_theta = self.theta.size
        w = self._pair_share(self.theta, n_a)
        x = np.cos(self.theta)
        P = np.empty((self.lmax + 1, n_theta))
        P[0] = 1.0
        if self.lmax >= 1:
            P[1] = x
        for l in range(1, self.lmax):
            P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
        self._P = P
        self.K = 2.0 * math.pi * P * (w * np.sin(self.theta) * wt)[None, :]

    def _pair_share(self, theta, n_a):
        tc = self.theta_c
        if tc >= math.pi:
            return np.ones_like(theta)
        v, wv = np.polynomial.legendre.leggauss(n_a)
        sv, wv = 0.5 * (v + 1.0), 0.5 * wv                      # s in (0, 1)
        a0 = np.abs(tc - theta)[:, None]
        a = a0 + (tc - a0) * sv[None, :] ** 2
        wa = wv[None, :] * 2.0 * (tc - a0) * sv[None, :] * np.sin(a)
        st, ct = np.sin(theta)[:, None], np.cos(theta)[:, None]
        c = (math.cos(tc) - np.cos(a) * ct) / (np.sin(a) * st)
        arc = np.arccos(np.clip(c, -1.0, 1.0)) / math.pi
        inner = np.where(theta < tc, 1.0 - np.cos(tc - theta), 0.0)   # rings wholly inside
        # solid angle of first points x in-cap share of their ring, over 4 pi
        return 2.0 * math.pi * (inner + (arc * wa).sum(axis=1)) / (4.0 * math.pi)

    def of_xi(self, xi_nodes):
        return self.K @ np.asarray(xi_nodes, dtype=np.float64)

    def of_cl(self, cl):
        cl = np.asarray(cl, dtype=np.float64)
        n = min(cl.size, self.lmax + 1)
        l = np.arange(n)
        xi = ((2 * l + 1) * cl[:n]) @ self._P[:n] / (4.0 * math.pi)
        if cl.size > n:
            xi = xi + xi_sph(self.theta, np.concatenate([np.zeros(n), cl[n:]]))
        return self.of_xi(xi)

    def of_table(self, k, p, R):
        """For a tabulated P_inf on uniform nodes k (piecewise linear, eq. xiinfpinf), xi at
        the chord 2 R sin(theta / 2) of each node."""
        r = 2.0 * R * np.sin(0.5 * self.theta)
        return self.of_xi(xi_of_table(r, k, p))


def band_deviation(a, b, lmin=2, width=10):
    """|sum_band a / sum_band b - 1| over bands [l0, l0 + width) from lmin to the last full band."""
    a, b = np.asarray(a), np.asarray(b)
    starts = np.arange(lmin, a.size - width + 1, width)
    sa = np.add.reduceat(a[lmin:starts[-1] + width], starts - lmin)
    sb = np.add.reduceat(b[lmin:starts[-1] + width], starts - lmin)
    return np.abs(sa / sb - 1.0)
