"""Harmonic analysis of cap maps: the recovered (pseudo-)C_l (test infrastructure only).

The paper judges simulated maps by the angular power spectrum they give back (Sec. III:
the recovered C_l of maps compared with the input). For maps sampled on rings of constant
colatitude (ring-major pixels, n_phi equally spaced azimuths phi_j = 2 pi j / n_phi per
ring) the spherical-harmonic coefficients are the quadrature

    a_lm = sum_rings dOmega_ring * lambda_lm(cos theta_ring) * sum_j T(ring, j) e^{-i m phi_j},

with lambda_lm(x) the orthonormal associated Legendre function (Y_lm = lambda_lm e^{i m phi},
Condon-Shortley phase) and dOmega_ring the solid angle per pixel. The pseudo-C_l of a real
map is (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1). On a cap (no mask correction) it is
the pseudo-spectrum, whose expectation the inversion oracle's ``cap_pseudo_cl`` gives.

lambda_lm comes from the standard three-term recurrence in l at fixed m, started from
lambda_mm = (-1)^m sqrt((2m+1)/(4 pi) prod_{i<=m} (2i-1)/(2i)) (1 - x^2)^{m/2}; the tests
pin it to SciPy's spherical harmonics.
"""
import math

import numpy as np


def legendre_lambda(m, lmax, x):
    """lambda_lm(x) for l = m .. lmax, shape (lmax - m + 1, len(x)), FP64."""
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    lam_mm = np.full_like(x, 1.0 / math.sqrt(4 * math.pi))
    for i in range(1, m + 1):
        lam_mm = -math.sqrt((2 * i + 1) / (2 * i)) * s * lam_mm
    out = np.zeros((lmax - m + 1, x.size))
    out[0] = lam_mm
    if lmax > m:
        out[1] = x * math.sqrt(2 * m + 3) * lam_mm
    for l in range(m + 2, lmax + 1):
        a = math.sqrt((4 * l * l - 1) / (l * l - m * m))
        a_prev = math.sqrt((4 * (l - 1) ** 2 - 1) / ((l - 1) ** 2 - m * m))
        out[l - m] = a * (x * out[l - 1 - m] - out[l - 2 - m] / a_prev)
    return out


def ring_alm(maps, cos_theta, n_phi, lmax, d_omega, mmax=None):
    """a_lm (n_maps, lmax + 1, mmax + 1), complex128, of ring-major maps
    (n_maps, n_ring * n_phi); entries with m > l are zero. d_omega is the solid angle of a
    pixel, a scalar or one value per ring. mmax defaults to min(lmax, n_phi // 2) (higher
    m alias on n_phi azimuths)."""
    maps = np.atleast_2d(np.asarray(maps, dtype=np.float64))
    cos_theta = np.asarray(cos_theta, dtype=np.float64)
    n_ring = cos_theta.size
    if mmax is None:
        mmax = min(lmax, n_phi // 2)
    F = np.fft.rfft(maps.reshape(maps.shape[0], n_ring, n_phi), axis=2)  # sum_j T e^{-i m phi_j}, m <= n_phi / 2
    # (m, map, ring) for m <= mmax, times the solid angle of each ring's pixels
    F = np.ascontiguousarray(np.moveaxis(F[:, :, : mmax + 1], 2, 0)) * np.broadcast_to(
        np.asarray(d_omega, dtype=np.float64), (n_ring,))[None, None, :]
    Fr, Fi = np.ascontiguousarray(F.real), np.ascontiguousarray(F.imag)
    alm = np.zeros((maps.shape[0], lmax + 1, mmax + 1), dtype=np.complex128)
    for m in range(mmax + 1):
        lam = legendre_lambda(m, lmax, cos_theta)                      # (lmax - m + 1, n_ring)
        alm[:, m:, m] = Fr[m] @ lam.T + 1j * (Fi[m] @ lam.T)
    return alm


def pseudo_cl(alm):
    """Pseudo-C_l (n_maps, lmax + 1) of real maps from their a_lm."""
    p = np.abs(alm) ** 2
    tot = p[:, :, 0] + 2.0 * p[:, :, 1:].sum(axis=2)
    l = np.arange(alm.shape[1])
    return tot / (2 * l + 1)


def band_ratio(cl_a, cl_b, lmin=2, width=10):
    """sum C_a / sum C_b - 1 over bands [l0, l0 + width) from lmin up to the last full band."""
    out = []
    for l0 in range(lmin, cl_a.size - width + 1, width):
        out.append(cl_a[l0:l0 + width].sum() / cl_b[l0:l0 + width].sum() - 1.0)
    return np.array(out)


def band_sums(cl, lmin=2, width=10):
    """sum of C_l over the bands [l0, l0 + width) from lmin up to the last full band; for an
    array of spectra (..., lmax + 1) the bands run over the last axis."""
    cl = np.asarray(cl, dtype=np.float64)
    starts = range(lmin, cl.shape[-1] - width + 1, width)
    return np.stack([cl[..., l0:l0 + width].sum(axis=-1) for l0 in starts], axis=-1)
