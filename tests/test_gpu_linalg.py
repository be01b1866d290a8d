"""FP64 Cholesky, whitening solve and their matrix-core product kernel on the GPU (the
covariance test of Sec. III B) against NumPy/SciPy and ``oracle.validation``.

Bars: the product kernel C -= A B^T within 1e-13 of max|C| (FP64 products, sums of at
most 64 terms); the factor of Gamma + s^2 I and the whitened maps within 1e-10 of their
largest entry (the factorisation's backward error is about n eps kappa^{1/2} per entry;
kappa <= 1e5 after the shift). Sizes span ragged tiles (1 .. 777) and several panels.
"""
import math

import numpy as np
import pytest

from oracle import healpix as ohp
from oracle import validation as oval

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cmbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx as c
    c.lib()
    return c


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("m,n,k,lower", [(1, 1, 1, 0), (64, 64, 64, 0), (65, 130, 7, 0), (200, 77, 64, 0),
                                         (150, 150, 33, 1), (777, 777, 64, 1)])
def test_gemm_nt_sub(cmbx, m, n, k, lower):
    rng = np.random.default_rng(m * 1000 + n + k)
    A = rng.standard_normal((m, k))
    B = A if (lower and m == n) else rng.standard_normal((n, k))
    C = rng.standard_normal((m, n))
    Ad, Bd, Cd = _dev(A), _dev(B), _dev(C)   # held until the kernel has run
    s = torch.cuda.current_stream().cuda_stream
    rc = cmbx.lib().cmbx_gemm_nt_sub(m, n, k, Ad.data_ptr(), k, Bd.data_ptr(), k, Cd.data_ptr(), n, lower, s)
    torch.cuda.synchronize()
    assert rc == 0
    got = Cd.cpu().numpy()
    want = C - A @ B.T
    if lower:
        low = np.tril(np.ones((m, n), dtype=bool))
        assert np.array_equal(got[~low], C[~low])   # the strict upper part untouched
        got, want = got[low], want[low]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.abs(want).max()


def _spd(n, seed, kappa=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.logspace(0, -math.log10(kappa), n)
    return (Q * w) @ Q.T


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 500])
def test_cholesky_random_spd(cmbx, n):
    A = _spd(n, n)
    Ad = _dev(A)
    info = cmbx.cholesky(Ad, shift=0.0)
    got = np.tril(Ad.cpu().numpy())
    want = np.linalg.cholesky(A)
    assert int(info.item()) == 0
    assert np.max(np.abs(got - want)) <= 1e-10 * np.abs(want).max()
    # the strict upper triangle is left as it was
    assert np.array_equal(np.triu(Ad.cpu().numpy(), 1), np.triu(A, 1))


@pytest.mark.parametrize("nside,theta,s2", [(8, 40.0, 1e-4), (16, 30.0, 1e-5), (32, 20.0, 1e-6)])
def test_cholesky_and_whiten_pixel_covariance(cmbx, nside, theta, s2):
    """Gamma of a HEALPix cap (device covariance kernel) plus s^2 I: the device factor and
    the whitened maps against oracle.validation (NumPy Cholesky, SciPy triangular solve)."""
    l = np.arange(200)
    cl = np.where(l >= 2, 1.0 / (l * (l + 1.0)) * np.exp(-((l / 60.0) ** 2)), 0.0)
    z_min = math.cos(math.radians(theta))
    dirs = ohp.cap_directions(nside, z_min)
    dirs_d = cmbx.healpix_cap(nside, z_min)
    G = cmbx.pixel_covariance(dirs_d, cl)
    n = G.shape[0]
    g_cpu = G.cpu().numpy()
    scale = g_cpu[0, 0]
    info = cmbx.cholesky(G, shift=s2 * scale)
    assert int(info.item()) == 0
    L = np.tril(G.cpu().numpy())
    want = np.linalg.cholesky(oval.pixel_covariance(dirs, cl) + s2 * scale * np.eye(n))
    assert np.max(np.abs(L - want)) <= 1e-10 * np.abs(want).max(), n
    rng = np.random.default_rng(nside)
    maps = rng.standard_normal((37, n)) * math.sqrt(scale)
    md = _dev(maps)
    cmbx.whiten(G, md)
    x = md.cpu().numpy()
    ref = oval.whiten(maps, oval.pixel_covariance(dirs, cl), noise_var=s2 * scale)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.abs(ref).max()


def test_cholesky_reports_non_positive_pivot(cmbx):
    A = _spd(100, 3)
    A[70, 70] = -1.0          # not positive definite: a pivot at or before column 71 fails
    Ad = _dev(A)
    info = cmbx.cholesky(Ad)
    col = int(info.item())
    assert 1 <= col <= 71
    # the next factorisation on the stream starts from a clear word
    info2 = cmbx.cholesky(_dev(_spd(100, 4)))
    assert int(info2.item()) == 0


def test_linalg_argument_errors(cmbx):
    L = cmbx.lib()
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert L.cmbx_cholesky(None, 4, 4, 0.0, None, None) == cmbx.EINVAL
    assert L.cmbx_cholesky(x.data_ptr(), 2, 1, 0.0, None, None) == cmbx.EINVAL
    assert L.cmbx_whiten(x.data_ptr(), 2, 2, x.data_ptr(), 0, 2, None) == cmbx.EINVAL
    assert L.cmbx_gemm_nt_sub(1, 1, 65, x.data_ptr(), 65, x.data_ptr(), 65, x.data_ptr(), 1, 0, None) == cmbx.EINVAL
