"""Pins of the oracle's half grid and inverse DFT: brute force, closed forms, symmetry."""
import numpy as np
import pytest

from oracle import field, noise, spectrum
from paper_2507_15703_amd import workloads


def _table(N, L=1.0):
    return workloads.powerlaw_cutoff_table(N, L, kc_modes=N / 4)


def _brute_force(h):
    """T(j) = sum_f T(f) exp(+2 pi i f.j / N) over the full grid, by direct summation."""
    N = h.shape[0]
    full = noise.full_grid(h.astype(np.complex128)).reshape(-1)
    idx = np.indices((N, N, N)).reshape(3, -1).T
    out = np.empty(N**3, dtype=np.complex128)
    for s in range(0, N**3, 512):
        ph = idx[s:s + 512] @ idx.T                      # f.j, integer
        out[s:s + 512] = np.exp(2j * np.pi * (ph % N) / N) @ full
    return out.reshape(N, N, N)


@pytest.mark.parametrize("N", [8, 12, 16])
def test_field_matches_brute_force_dft(N):
    k, p = _table(N)
    h = noise.halfgrid(N, 1.0, 3, k, p)
    bf = _brute_force(h)
    f = field.field(h)
    rms = np.sqrt(np.mean(f**2))
    assert np.max(np.abs(bf.imag)) <= 1e-13 * rms       # Hermitian: the full sum is real
    assert np.max(np.abs(bf.real - f)) <= 1e-13 * rms


@pytest.mark.parametrize("N", [8, 24])
def test_hermitian_planes(N):
    k, p = _table(N)
    for dt in (np.float64, np.float32):
        h = noise.halfgrid(N, 1.0, 11, k, p, dtype=dt)
        for iz in (0, N // 2):
            pl = h[:, :, iz]
            mir = pl[(-np.arange(N)) % N][:, (-np.arange(N)) % N]
            assert np.array_equal(pl, np.conj(mir))     # exact conjugate pairs
            for ix in (0, N // 2):
                for iy in (0, N // 2):
                    assert pl[ix, iy].imag == 0.0
        assert h[0, 0, 0] == 0                           # k = 0 carries no power


def test_single_mode_closed_form():
    # One mode f and its mirror: T(j) = 2 A cos(2 pi f.j / N + phi).
    N = 12
    h = np.zeros((N, N, N // 2 + 1), dtype=np.complex128)
    A, phi = 0.7, 0.4
    h[2, 11, 3] = A * np.exp(1j * phi)
    t = field.field(h)
    j = np.indices((N, N, N))
    ref = 2 * A * np.cos(2 * np.pi * (2 * j[0] - 1 * j[1] + 3 * j[2]) / N + phi)
    assert np.max(np.abs(t - ref)) < 1e-14


def test_parseval():
    N = 16
    k, p = _table(N)
    h = noise.halfgrid(N, 1.0, 5, k, p)
    t = field.field(h)
    full = noise.full_grid(h)
    assert np.sum(t**2) == pytest.approx(N**3 * np.sum(np.abs(full) ** 2), rel=1e-12)


def test_mode_variance_is_p_box():
    # E|T(f)|^2 = P_box(|f|) for generic and self-conjugate modes (eq. pboxxi), checked
    # over realisations on the modes of one shell.
    N = 8
    L = 2.0
    k, p = workloads.gaussian_table(L, 1.0, 0.3)
    pbox = spectrum.p_box_table(N, L, k, p)
    m = spectrum.mode_m(N)
    acc = np.zeros(m.shape)
    nreal = 400
    for s in range(nreal):
        acc += np.abs(noise.halfgrid(N, L, 100 + s, k, p)) ** 2
    ratio = acc / nreal / np.where(pbox[m] > 0, pbox[m], 1)
    gen = np.ones(m.shape, bool)
    gen[:, :, [0, N // 2]] = False
    sc = np.zeros(m.shape, bool)
    for ix in (0, N // 2):
        for iy in (0, N // 2):
            sc[ix, iy, [0, N // 2]] = True
    sc[0, 0, 0] = False
    # generic: |T|^2 / P ~ chi2_2 / 2 (sd 1/sqrt(n)); self-conjugate: chi2_1 (sd sqrt(2/n))
    assert abs(ratio[gen].mean() - 1) < 5 / np.sqrt(nreal * gen.sum())
    assert np.all(np.abs(ratio[sc] - 1) < 6 * np.sqrt(2 / nreal))


def test_field_variance_is_lattice_xi0():
    # The paper's xi(0) test: <T^2> over the box equals sum_f P_box (eq. pboxxi at r = 0).
    N, L = 16, 1.0
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=4)
    xi0 = spectrum.lattice_xi0(N, L, k, p)
    vals = [np.mean(field.field(noise.halfgrid(N, L, s, k, p)) ** 2) for s in range(40)]
    assert np.mean(vals) == pytest.approx(xi0, rel=4 * np.std(vals) / np.sqrt(40) / xi0)


def test_zero_weight_modes_are_exactly_zero():
    # a table that ends below the largest lattice |k|: every mode beyond it is +0 (its
    # conjugate partner on the planes iz = 0, N/2 is 0 - 0i), every mode inside is drawn
    N, L = 16, 1.0
    k = np.linspace(0.0, 2 * np.pi * 6, 40)
    p = np.exp(-k / 30.0)
    h = noise.halfgrid(N, L, 7, k, p, dtype=np.float32)
    m = spectrum.mode_m(N)
    kk = 2 * np.pi / L * np.sqrt(m)
    outside = kk > k[-1]
    assert np.all(h.real[outside] == 0) and np.all(h.imag[outside] == 0)
    gen = outside.copy()
    gen[:, :, 0] = gen[:, :, N // 2] = False                       # generic modes: +0 exactly
    assert not np.any(np.signbit(h.real[gen])) and not np.any(np.signbit(h.imag[gen]))
    inside = (~outside) & (m > 0)
    assert np.all(np.abs(h[inside]) > 0)
