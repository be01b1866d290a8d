"""Pins of the flat-box and 2-D (hybrid) method oracle (``oracle.slab``), CPU only.

* eq. finalpbox: with M = N and dp = L / N the flat P_box is the cubic one.
* The flat 3-D field against the brute-force inverse DFT over the whole N x N x M lattice
  (8 x 8 x 4, 8 x 8 x 6): the half grid's Hermitian rules, the axes and the sign.
* The hybrid column covariance against eq. pboxxi: the covariance of the layers implied
  by Gamma, transformed back over (k_x, k_y), equals the 3-D lattice correlation
  sum_k P_box e^{i k.r} of the N x N x M box at every separation within the layers.
* The symmetric root: S S^T = Gamma, S = S^T, and a Cholesky factor of a positive definite
  Gamma gives the same Gamma.
* Statistics of the generator: the empirical covariance of hybrid columns over 4000 seeds
  is Gamma (chi^2), and in the h = M limit the hybrid maps' empirical pixel covariance is
  the 3-D method's exact pixel covariance on the same flat box.
* The sizing rule of Sec. II C, by hand for one case.
"""
import math

import numpy as np
import pytest

from oracle import gather as ogather
from oracle import slab
from oracle import spectrum as ospec


def _gauss(dp, fc_cells, n=2000):
    """P_inf = exp(-(k / k_c)^2), k_c = 2 pi / (fc_cells dp), on [0, 2.5 k_c ... beyond the box's band]."""
    kc = 2 * math.pi / (fc_cells * dp)
    k = np.linspace(0.0, 6.0 * kc, n)
    return k, np.exp(-((k / kc) ** 2))


def test_flat_p_box_reduces_to_cubic():
    N, L = 16, 1.7
    k, p = _gauss(L / N, 4.0)
    flat = slab.p_box_flat(N, N, L / N, k, p)
    cubic = ospec.p_box_table(N, L, k, p)
    s = np.arange(flat.shape[0])[:, None]
    fz = np.arange(flat.shape[1])[None, :]
    assert np.allclose(flat, cubic[s + fz * fz], rtol=1e-13, atol=0)


@pytest.mark.parametrize("N,M", [(8, 4), (8, 6)])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_flat_field_brute_force(N, M, dt):
    dp = 0.11
    k, p = _gauss(dp, 2.5)
    h = slab.flat_halfgrid(N, M, dp, 7, k, p, dtype=dt)
    got = slab.flat_layers(h)                    # [z][x][y]
    full = slab.flat_full_grid(h.astype(np.complex128))   # [fx][fy][fz] array indices
    x = np.arange(N)
    z = np.arange(M)
    ex = np.exp(2j * np.pi * np.outer(x, x) / N)  # [index][position]
    ez = np.exp(2j * np.pi * np.outer(z, z) / M)
    want = np.einsum("abc,ai,bj,ck->kij", full, ex, ex, ez)
    assert np.max(np.abs(want.imag)) <= 1e-13 * np.sqrt(np.mean(want.real**2))
    assert np.allclose(got, want.real, rtol=0, atol=1e-12 * np.abs(want.real).max())
    # Parseval: sum of squares of the field = N^2 M sum over the lattice of |T|^2
    assert np.sum(got**2) == pytest.approx(N * N * M * np.sum(np.abs(full) ** 2), rel=1e-12)


def test_flat_halfgrid_conjugate_rules():
    N, M, dp = 8, 6, 0.2
    k, p = _gauss(dp, 3.0)
    h = slab.flat_halfgrid(N, M, dp, 11, k, p)
    for iy in (0, N // 2):
        for ix in range(N):
            for iz in range(M):
                assert h[ix, iy, iz] == np.conj(h[(-ix) % N, iy, (-iz) % M])
    # the eight self-conjugate modes are real; the k = 0 mode is zero
    for ix in (0, N // 2):
        for iy in (0, N // 2):
            for iz in (0, M // 2):
                assert h[ix, iy, iz].imag == 0
    assert h[0, 0, 0] == 0


def _lattice_xi(N, M, dp, k, p):
    """3-D lattice correlation of the flat box at every separation [dz][dx][dy] (eq. pboxxi)."""
    pb = slab.p_box_flat(N, M, dp, k, p)
    f = np.minimum(np.arange(N), N - np.arange(N))
    fz = np.minimum(np.arange(M), M - np.arange(M))
    P = pb[(f[:, None] ** 2 + f[None, :] ** 2)[:, :, None], fz[None, None, :]]   # [fx][fy][fz]
    xi = np.fft.ifftn(P) * P.size
    return np.transpose(xi.real, (2, 0, 1))


@pytest.mark.parametrize("N,M,h", [(16, 8, 5), (12, 12, 12)])
def test_hybrid_gamma_is_the_lattice_correlation(N, M, h):
    dp = 0.07
    k, p = _gauss(dp, 3.0)
    xi = slab.column_xi(N, M, dp, k, p, h)                  # [s][dz]
    f = np.minimum(np.arange(N), N - np.arange(N))
    s = f[:, None] ** 2 + f[None, :] ** 2
    per_col = xi[s]                                          # [fx][fy][dz]
    implied = np.fft.ifftn(per_col, axes=(0, 1)) * (N * N)   # back over (k_x, k_y)
    implied = np.transpose(implied.real, (2, 0, 1))          # [dz][dx][dy]
    want = _lattice_xi(N, M, dp, k, p)[:h]
    assert np.allclose(implied, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_symmetric_root():
    N, M, h, dp = 16, 16, 7, 0.05
    k, p = _gauss(dp, 2.0)
    xi = slab.column_xi(N, M, dp, k, p, h)
    S = slab.hybrid_factors(N, M, h, dp, k, p)
    for s in (0, 1, 2, 5, 13, 128):
        G = slab.gamma(xi[s])
        assert np.allclose(S[s], S[s].T, atol=0)
        assert np.allclose(S[s] @ S[s].T, G, rtol=0, atol=1e-12 * np.abs(G).max())
    # a positive definite Gamma: its Cholesky factor gives the same covariance
    G = slab.gamma(xi[5]) + 1e-3 * xi[5][0] * np.eye(h)
    L = np.linalg.cholesky(G)
    R = slab.sym_sqrt(G)
    assert np.allclose(L @ L.T, R @ R.T, rtol=0, atol=1e-12 * G.max())


def test_hybrid_column_covariance_statistics():
    """Empirical covariance of the columns (ix, iy) = (3, 2) and (0, 0) over 4000 seeds is
    Gamma: E[T T^H] = Gamma for the generic column, E[T T^T] = 0 (circular) and E[T T^T] =
    Gamma for the real one. chi^2 per entry with the empirical variances."""
    N, M, h, dp = 8, 16, 4, 0.1
    k, p = _gauss(dp, 2.0)
    xi = slab.column_xi(N, M, dp, k, p, h)
    n = 4000
    cols = np.stack([slab.hybrid_columns(N, M, h, dp, s, k, p) for s in range(n)])   # (n, h, N, N/2+1)
    for (ix, iy, real) in ((3, 2, False), (0, 0, True), (2, 0, False)):
        v = cols[:, :, ix, iy]
        G = slab.gamma(xi[ix * ix + iy * iy])
        prod = np.einsum("ni,nj->nij", v, v.conj())
        m, e = prod.mean(0), prod.std(0) / math.sqrt(n)
        z = np.abs(m.real - G) / np.maximum(e.real, 1e-300)
        assert z.max() < 4.5, (ix, iy, z.max())
        if real:
            assert np.all(v.imag == 0)
        else:
            pseudo = np.einsum("ni,nj->nij", v, v).mean(0)
            assert np.max(np.abs(pseudo)) < 5 * np.max(np.abs(e)) + 1e-12


def _pixel_cov_3d(N, M, dp, k, p, dirs, r, obs, interp):
    """Exact pixel covariance of the 3-D method on the flat box: sum_ab w_ia w_jb xi(x_a - x_b)."""
    xi = _lattice_xi(N, M, dp, k, p)                          # [dz][dx][dy], periodic
    pos = slab.positions(dp, r, dirs, obs)
    i0 = np.floor(pos)
    f = pos - i0
    offs = np.arange(-1, 3) if interp == "tricubic" else np.arange(0, 2)
    kern = ogather.keys_kernel if interp == "tricubic" else ogather.linear_kernel
    w = kern(offs[None, None, :] - f[:, :, None])            # (n, 3, K)
    idx = i0[:, :, None].astype(np.int64) + offs[None, None, :]
    K = offs.size
    n = dirs.shape[0]
    W = np.einsum("na,nb,nc->nabc", w[:, 0], w[:, 1], w[:, 2]).reshape(n, -1)
    X = np.stack(np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij"), -1).reshape(-1, 3)
    node = np.stack([idx[:, 0][:, X[:, 0]], idx[:, 1][:, X[:, 1]], idx[:, 2][:, X[:, 2]]], -1)   # (n, K^3, 3)
    C = np.zeros((n, n))
    for i in range(n):
        d = node[i][:, None, None, :] - node[None, :, :, :]   # (K^3, n, K^3, 3)
        val = xi[d[..., 2] % M, d[..., 0] % N, d[..., 1] % N]
        C[i] = np.einsum("a,anb,nb->n", W[i], val, W)
    return C


def test_hybrid_h_equals_m_limit_matches_3d_pixel_covariance():
    """With h = M the layers are the whole flat box: the hybrid maps' empirical pixel
    covariance (3000 seeds) matches the 3-D method's exact pixel covariance (chi^2), and so
    do the flat 3-D method's own maps."""
    N, M, dp, r = 8, 8, 0.1, 0.25
    k, p = _gauss(dp, 2.2)
    rng = np.random.default_rng(4)
    d = rng.standard_normal((6, 3))
    dirs = d / np.linalg.norm(d, axis=1, keepdims=True)
    obs = slab.default_observer(N, M, dp)
    C = _pixel_cov_3d(N, M, dp, k, p, dirs, r, obs, "tricubic")
    n = 3000
    for kind in ("hybrid", "flat"):
        maps = np.empty((n, dirs.shape[0]))
        for s in range(n):
            if kind == "hybrid":
                lay = slab.hybrid_layers(slab.hybrid_columns(N, M, M, dp, s, k, p))
            else:
                lay = slab.flat_layers(slab.flat_halfgrid(N, M, dp, s, k, p))
            maps[s] = slab.gather_layers(lay, dp, r, dirs, "tricubic", obs, periodic_z=True)
        prod = np.einsum("ni,nj->nij", maps, maps)
        m, e = prod.mean(0), prod.std(0) / math.sqrt(n)
        z = np.abs(m - C) / e
        assert z.max() < 4.5, (kind, z.max())


def test_gather_layers_reproduces_nodes_and_flags_outside():
    N, nz, dp = 8, 6, 0.1
    rng = np.random.default_rng(1)
    lay = rng.standard_normal((nz, N, N))
    obs = np.array([0.4, 0.4, 0.2])
    dirs = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    down = np.array([[0.0, 0.0, -1.0]])
    for interp in ("trilinear", "tricubic"):
        v = slab.gather_layers(lay, dp, 0.1, dirs, interp, obs, periodic_z=False)
        # nodes (x, y, z) = (4, 4, 3) and (5, 4, 2)
        assert v[0] == pytest.approx(lay[3, 4, 4], abs=1e-14) and v[1] == pytest.approx(lay[2, 5, 4], abs=1e-14)
        # z = 0.5 cells: the tricubic stencil reaches z = -1, outside the layers
        v = slab.gather_layers(lay, dp, 0.15, down, interp, obs, periodic_z=False)
        assert np.isnan(v[0]) == (interp == "tricubic")
        vp = slab.gather_layers(lay, dp, 0.15, down, interp, obs, periodic_z=True)
        assert np.isfinite(vp[0])


def test_box_size_rule():
    # b = 0.01 rad, theta = 15 deg on the unit sphere: dp = 0.85 * 0.002 = 0.0017;
    # width 2 sin 15 / dp = 304.5 points -> 2x = 609 -> 1024; height (1 - cos 15)/dp = 20.07 -> 2x -> 64
    N, M, dp = slab.box_size(0.01, math.radians(15.0))
    assert (N, M) == (1024, 64) and dp == pytest.approx(0.0017)
    N2, M2, _ = slab.box_size(0.01, math.radians(15.0), size_factor=0.25)
    assert (N2, M2) == (256, 16)   # Table I's row for these b and theta (N = 256, M = 16)
