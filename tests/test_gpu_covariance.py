"""HIP pixel covariance (Sec. III B, eq. harmonics) against the oracle.

Both sides sum the same series in FP64, the oracle with SciPy's Legendre polynomials, the
kernel by the three-term recurrence; the bar, max|dGamma| <= 1e-12 max|Gamma|, bounds
the recurrence's rounding (about l ulp) for l up to 700. Sizes span several 16 x 16 tiles
with ragged edges.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx
    return cmbx, torch


def _cl(lmax, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.2, 1.0, lmax + 1) / (1.0 + np.arange(lmax + 1)) ** 1.5


@pytest.mark.parametrize("nside,theta,lmax", [(1, 180.0, 0), (2, 90.0, 1), (4, 60.0, 2), (8, 40.0, 50),
                                              (16, 25.0, 300), (32, 12.0, 700), (64, 8.0, 120)])
def test_covariance_matches_oracle(env, nside, theta, lmax):
    cmbx, torch = env
    from oracle import healpix as hp
    from oracle import validation as ov
    z_min = math.cos(math.radians(theta))
    dirs_h = hp.cap_directions(nside, z_min)
    cl = _cl(lmax, nside)
    print(f"[cov] nside={nside} n={len(dirs_h)} lmax={lmax}", flush=True)
    got = cmbx.pixel_covariance(torch.tensor(dirs_h, device="cuda"), cl)
    torch.cuda.synchronize()
    ref = ov.pixel_covariance(dirs_h, cl)
    err = np.max(np.abs(got.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err


def test_covariance_into_larger_buffer(env):
    cmbx, torch = env
    from oracle import healpix as hp
    from oracle import validation as ov
    dirs_h = hp.cap_directions(8, math.cos(math.radians(30.0)))
    n = len(dirs_h)
    out = torch.full((n + 3, n), 5.0, dtype=torch.float64, device="cuda")
    cmbx.pixel_covariance(torch.tensor(dirs_h, device="cuda"), _cl(20, 1), out=out)
    torch.cuda.synchronize()
    flat = out.view(-1).cpu().numpy()
    np.testing.assert_allclose(flat[: n * n].reshape(n, n), ov.pixel_covariance(dirs_h, _cl(20, 1)),
                               rtol=0, atol=1e-13)
    assert np.all(flat[n * n:] == 5.0)  # nothing written past n^2
