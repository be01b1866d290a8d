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
    # A P for the samples P(k_j) of a Gaussian P_inf is eq. xiinfpinf for the table read
    # as linear between nodes: within the interpolation error of the Gaussian, |P_lin - P|
    # <= dk^2 max|P''| / 8, of its closed-form correlation.
    amp, s = 2.0, 0.02
    cl = workloads.synthetic_cl(300)
    r, b, k, A, c = oinv.programme(cl, 0.45, math.radians(30), 1 / 180.0, k_max=12 / s)
    p = amp * np.exp(-0.5 * (k * s) ** 2)
    ref = oinv.xi_inf_gaussian(r, amp, s)
    dk = k[1] - k[0]
    # bound: sum over intervals of dk^2 / 8 max|P''| x 4 pi int k^2 dk, max|P''| sampled
    # finely on each interval; plus the tail beyond the table (P_lin = 0 there)
    u = np.linspace(0.0, 1.0, 65)
    q = k[:-1, None] + dk * u[None, :]
    d2 = amp * s**2 * np.abs((q * s) ** 2 - 1.0) * np.exp(-0.5 * (q * s) ** 2)
    shell = 4 * math.pi * (k[1:] ** 3 - k[:-1] ** 3) / 3
    tail = 4 * math.pi * amp * (k[-1] ** 2 / s) * np.exp(-0.5 * (k[-1] * s) ** 2) * 4
    bound = float(np.sum(dk**2 / 8 * d2.max(axis=1) * shell)) + tail
    assert bound < 5e-3 * ref[0]
    assert np.max(np.abs(A @ p - ref)) <= bound
    assert np.allclose(c, A.sum(axis=0))


@pytest.mark.parametrize("R,theta", [(0.45, 30.0), (1.0, 20.0)])
def test_programme_matrix_is_the_integral_of_the_linear_table(R, theta):
    """For any table, A x is eq. xiinfpinf of the piecewise-linear P_inf through it (zero
    beyond the last node): against SciPy's adaptive quadrature of that integral, with the
    nodes as break points, at chords across the cap."""
    import scipy.integrate
    import scipy.special
    cl = workloads.synthetic_cl(200)
    r, b, k, A, c = oinv.programme(cl, R, math.radians(theta), 1 / 120.0, k_max=200.0 / R)
    x = np.random.default_rng(5).uniform(0.0, 1.0, k.size) * np.exp(-k / k[-1] * 3)
    x[0] = 0.0
    x[k.size // 2] = 0.0           # a zero node in the middle: its neighbours' hats end there

    def integrand(q, rr):
        return 4 * math.pi * q * q * scipy.special.spherical_jn(0, q * rr) * np.interp(q, k, x)

    for i in (0, 1, r.size // 3, r.size - 1):
        want = 0.0
        for j in range(k.size - 1):   # interval by interval: the integrand is smooth on each
            want += scipy.integrate.quad(integrand, k[j], k[j + 1], args=(r[i],), epsabs=0, epsrel=1e-13)[0]
        assert (A @ x)[i] == pytest.approx(want, rel=1e-11, abs=1e-13 * abs(want) + 1e-300), i


def test_hat_masses_closed_form():
    # row r = 0: 4 pi int k^2 phi_j dk = 4 pi dk (k_j^2 + dk^2 / 6) for an interior node,
    # 4 pi dk (k_j^2 / 2 - k_j dk / 3 + dk^2 / 12) for the last (its rising half only)
    cl = workloads.synthetic_cl(100)
    r, b, k, A, c = oinv.programme(cl, 0.4, math.radians(25), 1 / 90.0, k_max=300.0)
    dk = k[1] - k[0]
    m = A[0]
    kj = k[1:-1]
    assert np.allclose(m[1:-1], 4 * math.pi * dk * (kj**2 + dk**2 / 6), rtol=1e-13)
    kl = k[-1]
    assert m[-1] == pytest.approx(4 * math.pi * dk * (kl**2 / 2 - kl * dk / 3 + dk**2 / 12), rel=1e-13)


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


@pytest.mark.parametrize("N,theta", [(128, 20.0), (256, 30.0)])
def test_box_variance_matches_programme(N, theta):
    """The programme's solution, sampled by the box (sum of P_box over the lattice, eq.
    finalpbox), carries the variance xi_sph(0) it was fitted to: within 1 % (the lattice's
    Riemann sum of the integral and the box's missing k = 0 mode). This ties the
    programme's quadrature to the box's reading of the table (linear between nodes)."""
    from oracle import spectrum as ospec
    L, rr = 1.0, 0.45
    lmax = workloads.lmax_for(N, L, rr)
    cl = workloads.synthetic_cl(lmax)
    r, b, k, A, c = oinv.programme(cl, rr, math.radians(theta), 1.0 / (0.6 * lmax), math.pi * N / L)
    _, x = oinv.solve(A, b, c)
    assert (A @ x)[0] == pytest.approx(b[0], rel=1e-5)
    assert ospec.lattice_xi0(N, L, k, x) == pytest.approx(b[0], rel=1e-2)
