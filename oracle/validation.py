"""The paper's covariance test of partial-sky maps (test infrastructure only).

Sec. III B: maps made from a power spectrum C_l are Gaussian with zero mean, so their
statistics are fixed by the pixel covariance, which eq. harmonics gives for every pair of
pixels from the angle between them:

    Gamma_ij = sum_l (2l + 1) C_l P_l(n_i . n_j) / (4 pi).

With Gamma = L L^T (Cholesky), the whitened vector x = L^{-1} m of a map m has independent
unit normal entries, which the paper checks with a Kolmogorov-Smirnov test; white noise of
variance s^2 added to the maps enters as Gamma + s^2 I.

Written from those definitions with SciPy's Legendre polynomials, NumPy's Cholesky and
triangular solve, and SciPy's KS test as library steps.
"""
import math

import numpy as np
import scipy.linalg
import scipy.special
import scipy.stats


def pixel_covariance(dirs, cl):
    """Gamma (n_pix, n_pix) of unit directions dirs (n_pix, 3) for C_l, l = 0 .. len(cl) - 1."""
    d = np.asarray(dirs, dtype=np.float64)
    x = np.clip(d @ d.T, -1.0, 1.0)
    out = np.zeros_like(x)
    for l, c in enumerate(np.asarray(cl, dtype=np.float64)):
        if c != 0.0:
            out += (2 * l + 1) * c / (4.0 * math.pi) * scipy.special.eval_legendre(l, x)
    return out


def whiten(maps, gamma, noise_var=0.0):
    """x = L^{-1} m for each map (rows of maps), Gamma + noise_var I = L L^T."""
    g = np.asarray(gamma, dtype=np.float64) + noise_var * np.eye(len(gamma))
    low = np.linalg.cholesky(g)
    m = np.atleast_2d(np.asarray(maps, dtype=np.float64))
    return scipy.linalg.solve_triangular(low, m.T, lower=True).T


def ks_unit_normal(x):
    """(statistic, p-value) of the KS test of all entries of x against N(0, 1)."""
    r = scipy.stats.kstest(np.ravel(x), "norm")
    return float(r.statistic), float(r.pvalue)
