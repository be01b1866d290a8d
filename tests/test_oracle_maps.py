"""Pins of the map harmonic analysis: SciPy's spherical harmonics, exact quadrature on
Gauss-Legendre rings, and the expected pseudo-C_l of the inversion oracle."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import maps as omaps


def _ylm(l, m, theta, phi):
    return scipy.special.sph_harm_y(l, m, theta, phi)


@pytest.mark.parametrize("m", [0, 1, 2, 7, 20])
def test_lambda_matches_scipy(m):
    th = np.linspace(0.01, math.pi - 0.01, 37)
    lam = omaps.legendre_lambda(m, 60, np.cos(th))
    for l in range(m, 61):
        ref = _ylm(l, m, th, 0.0).real
        assert np.allclose(lam[l - m], ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max())), l


def test_full_sky_gauss_legendre_recovers_alm():
    # A band-limited real map synthesised from random a_lm with SciPy's Y_lm is integrated
    # exactly by Gauss-Legendre rings with n_phi > 2 lmax azimuths.
    lmax, n_ring, n_phi = 12, 16, 32
    rng = np.random.default_rng(0)
    alm = rng.standard_normal((lmax + 1, lmax + 1)) + 1j * rng.standard_normal((lmax + 1, lmax + 1))
    alm[:, 0] = alm[:, 0].real
    alm[np.triu_indices(lmax + 1, 1)] = 0
    x, w = np.polynomial.legendre.leggauss(n_ring)
    th = np.arccos(x)[:, None]
    phi = (2 * math.pi * np.arange(n_phi) / n_phi)[None, :]
    T = np.zeros((n_ring, n_phi))
    for l in range(lmax + 1):
        T += (alm[l, 0] * _ylm(l, 0, th, phi)).real
        for m in range(1, l + 1):
            T += 2 * (alm[l, m] * _ylm(l, m, th, phi)).real
    got = omaps.ring_alm(T.ravel(), x, n_phi, lmax, w * 2 * math.pi / n_phi)[0]
    assert np.allclose(got, alm, rtol=0, atol=1e-12 * np.abs(alm).max())
    cl = omaps.pseudo_cl(got[None])[0]
    ref = (np.abs(alm[:, 0]) ** 2 + 2 * (np.abs(alm[:, 1:]) ** 2).sum(axis=1)) / (2 * np.arange(lmax + 1) + 1)
    assert np.allclose(cl, ref, rtol=1e-12)


def test_band_ratio():
    a = np.arange(1.0, 33.0)
    r = omaps.band_ratio(2 * a, a, lmin=2, width=10)
    assert r.shape == (3,) and np.allclose(r, 1.0)


def test_band_sums():
    a = np.arange(25.0)
    assert np.allclose(omaps.band_sums(a), [a[2:12].sum(), a[12:22].sum()])
    two = np.stack([a, 2 * a])
    assert np.allclose(omaps.band_sums(two)[1], 2 * omaps.band_sums(a))
