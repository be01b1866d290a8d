"""Pins of the inversion oracle (closed forms, planted solutions) and of the host inversion
against it."""
import math

import numpy as np
import pytest

from oracle import inversion as oinv
from paper_2507_15703_amd import spectrum as pspec
from paper_2507_15703_amd import workloads


def test_xi_sph_at_zero_and_recurrence():
    cl = workloads.synthetic_cl(200)
    ref0 = np.sum((2 * np.arange(cl.size) + 1) * cl) / (4 * math.pi)
    assert oinv.xi_sph([0.0], cl)[0] == pytest.approx(ref0, rel=1e-13)
    th = np.linspace(0, math.pi, 301)
    assert np.allclose(pspec.xi_sph(th, cl), oinv.xi_sph(th, cl), rtol=0, atol=1e-12 * ref0)


def test_gaussian_cl_closed_form_gives_sphere_restriction():
    # A 3-D Gaussian correlation restricted to a sphere of radius R: xi_sph(theta) must
    # equal xi_inf(chord(theta)) when C_l = 4 pi A e^{-x} i_l(x).
    amp, s, R = 1.7, 0.05, 0.45
    cl = oinv.cl_gaussian(400, amp, s, R)
    th = np.linspace(0, 0.6, 40)
    lhs = oinv.xi_sph(th, cl)
    rhs = amp * np.exp(-oinv.chord(th, R) ** 2 / (2 * s * s))
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-9 * amp)


def test_programme_matrix_integrates_gaussian():
    # A P_inf for a Gaussian P_inf is the Riemann sum of eq. xiinfpinf.
    amp, s = 2.0, 0.02
    cl = workloads.synthetic_cl(300)
    r, b, k, A, c = oinv.programme(cl, 0.45, math.radians(30), 1 / 180.0, k_max=12 / s)
    p = amp * np.exp(-0.5 * (k * s) ** 2)
    ref = oinv.xi_inf_gaussian(r, amp, s)
    assert np.allclose(A @ p, ref, rtol=0, atol=1e-6 * ref[0])
    assert np.allclose(c, A.sum(axis=0))


def test_lp_recovers_planted_feasible_problem():
    # b = A x_true with x_true >= 0: the optimum makes every constraint an equality,
    # with value sum(b) (eq. sumconstraint).
    rng = np.random.default_rng(3)
    cl = workloads.synthetic_cl(250)
    r, _, k, A, c = oinv.programme(cl, 0.45, math.radians(25), 1 / 150.0, k_max=600.0)
    x_true = np.zeros(k.size)
    x_true[1:] = rng.uniform(0, 1, k.size - 1) * np.exp(-k[1:] / 200.0) / (k[1:] ** 2)
    b = A @ x_true
    val, x = oinv.solve(A, b, c)
    assert val == pytest.approx(b.sum(), rel=1e-6)
    assert np.max(np.abs(A @ x - b)) <= 1e-6 * b[0]


def test_lp_homogeneous_in_cl():
    cl = workloads.synthetic_cl(150)
    r, b, k, A, c = oinv.programme(cl, 0.4, math.radians(20), 1 / 90.0, k_max=400.0)
    v1, x1 = oinv.solve(A, b, c)
    v2, x2 = oinv.solve(A, 3.0 * b, c)
    assert v2 == pytest.approx(3.0 * v1, rel=1e-6)


@pytest.mark.parametrize("N,theta", [(128, 20.0), (256, 30.0)])
def test_host_inversion_matches_oracle(N, theta):
    L, rr = 1.0, 0.45
    lmax = workloads.lmax_for(N, L, rr)
    cl = workloads.synthetic_cl(lmax)
    beam = 1.0 / (0.6 * lmax)
    k, p, info = pspec.invert(cl, rr, math.radians(theta), beam, N=N, L=L)
    r, b, k2, A, c = oinv.programme(cl, rr, math.radians(theta), beam, math.pi * N / L)
    assert np.allclose(k, k2, rtol=1e-14) and np.allclose(b, pspec.lp_problem(cl, rr, math.radians(theta), beam, math.pi * N / L)["b"], rtol=1e-12)
    val, _ = oinv.solve(A, b, c)
    # the optimal value is unique; the solution need not be
    assert c @ p == pytest.approx(val, rel=1e-5)
    assert np.min(A @ p - b) >= -1e-7 * b[0]
    assert np.all(p >= 0)


def test_cl_box_normalisation():
    # sum_l (2l+1) C_l^box / 4 pi = <T^2> = sum_f P_box (the xi(0) chain of the paper's tests)
    from oracle import spectrum as ospec
    N, L, R = 32, 1.0, 0.3
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=4)
    cl = oinv.cl_box(N, L, R, k, p, 200)
    lhs = np.sum((2 * np.arange(cl.size) + 1) * cl) / (4 * math.pi)
    assert lhs == pytest.approx(ospec.lattice_xi0(N, L, k, p), rel=1e-10)


def test_cap_pseudo_cl_full_sky_inverts_harmonics():
    cl = workloads.synthetic_cl(60)
    got = oinv.cap_pseudo_cl(lambda th: oinv.xi_sph(th, cl), math.pi, 60)
    assert np.allclose(got, cl, rtol=1e-8, atol=1e-8 * cl.max())


def test_cap_pair_weight_limits():
    # zero separation: every pair partner stays inside, w(0) = f_sky of the cap
    tc = math.radians(30)
    fsky = (1 - math.cos(tc)) / 2
    assert oinv.cap_pair_weight([1e-9], tc)[0] == pytest.approx(fsky, rel=1e-6)
    assert oinv.cap_pair_weight([2 * tc + 1e-6], tc)[0] == pytest.approx(0.0, abs=1e-12)
    # integral over the sphere of w equals f_sky^2 (ordered pairs)
    th = np.linspace(0, 2 * tc, 20001)
    integ = np.trapezoid(oinv.cap_pair_weight(th, tc) * 2 * math.pi * np.sin(th), th)
    assert integ == pytest.approx(4 * math.pi * fsky**2, rel=2e-3)


def test_xi_inf_of_matches_programme_rows():
    cl = workloads.synthetic_cl(120)
    r, b, k, A, c = oinv.programme(cl, 0.4, math.radians(20), 1 / 70.0, k_max=300.0)
    p = np.exp(-k / 60.0)
    assert np.allclose(oinv.xi_inf_of(k, p, r), A @ p, rtol=1e-12, atol=1e-12 * abs(A @ p).max())
