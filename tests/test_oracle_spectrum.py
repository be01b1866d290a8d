"""Pins of the box-spectrum tables (eq. finalpbox) against closed forms."""
import numpy as np
import pytest

from oracle import spectrum
from paper_2507_15703_amd import workloads


def test_interp_nodes_and_outside():
    k = np.array([0.5, 1.0, 2.0, 4.0])
    p = np.array([3.0, 2.0, 5.0, 1.0])
    assert list(spectrum.interp_p(k, p, k[:-1])) == list(p[:-1])
    assert spectrum.interp_p(k, p, [4.0])[0] == pytest.approx(1.0, abs=1e-15)
    assert list(spectrum.interp_p(k, p, [0.0, 0.49, 4.01, 100.0])) == [0.0] * 4
    assert spectrum.interp_p(k, p, [1.5])[0] == pytest.approx(3.5, rel=1e-15)
    assert spectrum.interp_p(k, p, [3.0])[0] == pytest.approx(3.0, rel=1e-15)


def test_p_box_normalisation_gaussian():
    # Continuum: xi_inf(0) = 4 pi int k^2 P dk = A (2 pi)^{3/2} / s^3 for P = A exp(-k^2 s^2 / 2).
    # The lattice sum of P_box = P_inf (2 pi / L)^3 must reproduce it (Riemann sum of a smooth,
    # well-resolved integrand), minus the k = 0 term A (2 pi / L)^3 that the box omits.
    A, s = 2.5, 0.05
    for L, N in [(1.0, 64), (2.0, 128)]:
        k, p = workloads.gaussian_table(L, A, s, n=20001)
        xi0 = spectrum.lattice_xi0(N, L, k, p)
        ref = A * (2 * np.pi) ** 1.5 / s**3 - A * (2 * np.pi / L) ** 3
        assert xi0 == pytest.approx(ref, rel=2e-6)


def test_weights_square_to_p_box():
    N, L = 32, 1.3
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=8)
    half, full = spectrum.weight_tables(N, L, k, p)
    pb = spectrum.p_box_table(N, L, k, p)
    assert half[0] == 0 and full[0] == 0
    assert np.allclose(2 * half**2, pb, rtol=1e-15, atol=0)
    assert np.allclose(full**2, pb, rtol=1e-15, atol=0)
    # the table passed covers every lattice |k|, so P_box is the formula at the nodes
    kk = spectrum.lattice_k(N, L)[1:]
    kc = 2 * np.pi * 8 / L
    ref = kk**-3 * np.exp(-((kk / kc) ** 2)) * (2 * np.pi / L) ** 3
    assert np.allclose(pb[1:], ref, rtol=1e-13)


def test_mode_m():
    N = 6
    m = spectrum.mode_m(N)
    assert m.shape == (6, 6, 4)
    assert m[0, 0, 0] == 0 and m[5, 1, 3] == 1 + 1 + 9 and m[3, 3, 3] == 27
