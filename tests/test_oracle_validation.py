"""Pins of the covariance-test oracle (Sec. III B, eq. harmonics).

The pixel covariance is checked against the addition theorem of spherical harmonics (the
sum over m of Y_lm(n_i) Y_lm(n_j)* built with SciPy's spherical harmonics, a route that
never evaluates a Legendre polynomial of the pair angle), its diagonal against the closed
form P_l(1) = 1, and positive semi-definiteness; the whitening and KS steps against exact
Gaussian draws with that covariance (accepted) and draws with the wrong scale (rejected).
"""
import math

import numpy as np
import pytest
import scipy.special

from oracle import healpix as hp
from oracle import validation as ov


def _sph_harm(m, l, theta, phi):
    # complex Y_lm with polar angle theta and azimuth phi
    if hasattr(scipy.special, "sph_harm_y"):
        return scipy.special.sph_harm_y(l, m, theta, phi)
    return scipy.special.sph_harm(m, l, phi, theta)


def _cl(lmax, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.2, 1.0, lmax + 1) / (1.0 + np.arange(lmax + 1)) ** 2


def test_covariance_equals_addition_theorem():
    dirs = hp.cap_directions(4, math.cos(math.radians(60.0)))
    cl = _cl(12)
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    ref = np.zeros((len(dirs), len(dirs)))
    for l, c in enumerate(cl):
        y = np.array([_sph_harm(m, l, theta, phi) for m in range(-l, l + 1)])  # (2l+1, n)
        ref += c * np.real(y.T @ np.conj(y))
    got = ov.pixel_covariance(dirs, cl)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * ref[0, 0])


def test_covariance_diagonal_and_psd():
    dirs = hp.cap_directions(8, math.cos(math.radians(25.0)))
    cl = _cl(40, seed=3)
    g = ov.pixel_covariance(dirs, cl)
    diag = sum((2 * l + 1) * c for l, c in enumerate(cl)) / (4 * math.pi)
    np.testing.assert_allclose(np.diag(g), diag, rtol=1e-13)
    np.testing.assert_array_equal(g, g.T)
    assert np.linalg.eigvalsh(g).min() > -1e-12 * diag


def test_whitened_exact_draws_pass_and_wrong_scale_fails():
    dirs = hp.cap_directions(8, math.cos(math.radians(30.0)))
    cl = _cl(30, seed=5)
    g = ov.pixel_covariance(dirs, cl)
    s2 = 1e-3 * g[0, 0]
    low = np.linalg.cholesky(g + s2 * np.eye(len(g)))
    rng = np.random.default_rng(11)
    z = rng.standard_normal((200, len(g)))
    maps = z @ low.T
    x = ov.whiten(maps, g, s2)
    np.testing.assert_allclose(x, z, rtol=0, atol=1e-9)
    stat, p = ov.ks_unit_normal(x)
    assert p > 1e-3
    stat_bad, p_bad = ov.ks_unit_normal(ov.whiten(1.1 * maps, g, s2))
    assert p_bad < 1e-6 and stat_bad > stat
