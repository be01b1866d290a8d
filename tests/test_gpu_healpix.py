"""HIP HEALPix cap pixels against the oracle (Sec. II D 1: the cap's pixels are the leading
pixels of a RING-ordered HEALPix map).

Ring heights are integer quotients taken the same way on both sides, so z and the pixel
count must be bit-exact; x and y go through FP64 sin/cos of the longitude (within a few
ulp of 1 on either side), bar 1e-15 absolute. One end-to-end map checks that the
directions drive the hot path like any others.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cmbx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx
    return cmbx, torch


def _compare(got, ref):
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got[:, 2], ref[:, 2])
    assert np.max(np.abs(got - ref)) <= 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 16, 63, 256])
def test_whole_sky_matches_oracle(n):
    cmbx, torch = _cmbx()
    from oracle import healpix as hp
    print(f"[healpix] whole sky nside={n}", flush=True)
    got = cmbx.healpix_cap(n, -1.0)
    torch.cuda.synchronize()
    _compare(got.cpu().numpy(), hp.all_pixels(n))


@pytest.mark.parametrize("n,theta_deg", [(2, 60.0), (16, 26.85), (64, 10.0), (512, 40.0), (2048, 26.85),
                                         (8192, 5.0)])
def test_caps_match_oracle(n, theta_deg):
    cmbx, torch = _cmbx()
    from oracle import healpix as hp
    z_min = math.cos(math.radians(theta_deg))
    print(f"[healpix] cap nside={n} theta={theta_deg}", flush=True)
    ref = hp.cap_directions(n, z_min)
    assert cmbx.healpix_cap_count(n, z_min) == ref.shape[0]
    got = cmbx.healpix_cap(n, z_min)
    torch.cuda.synchronize()
    _compare(got.cpu().numpy(), ref)


def test_cap_into_larger_buffer_and_ring_edge():
    cmbx, torch = _cmbx()
    from oracle import healpix as hp
    # z_min exactly at the polar zone's last ring (z = 2/3): that ring is in
    n = 12
    ref = hp.cap_directions(n, 2.0 / 3.0)
    assert ref.shape[0] == 2 * n * (n + 1)
    buf = torch.full((ref.shape[0] + 7, 3), 7.0, dtype=torch.float64, device="cuda")
    got = cmbx.healpix_cap(n, 2.0 / 3.0, out=buf)
    torch.cuda.synchronize()
    _compare(got.cpu().numpy(), ref)
    assert torch.all(buf[ref.shape[0]:] == 7.0)  # nothing written past the cap
    assert cmbx.healpix_cap(n, 1.5).shape == (0, 3)


def test_map_on_healpix_cap_matches_oracle():
    cmbx, torch = _cmbx()
    from oracle import field as ofield
    from oracle import gather as ogather
    from oracle import healpix as hp
    from oracle import noise as onoise
    from paper_2507_15703_amd import workloads
    N, L, r, seed = 32, 1.0, 0.4, 11
    k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=8)
    z_min = math.cos(math.radians(30.0))
    print("[healpix] map on nside 32 cap, N 32 f64", flush=True)
    dirs = cmbx.healpix_cap(32, z_min)
    plan = cmbx.Plan(N, L, "f64", batch=1, interp="tricubic")
    plan.spectrum_table(k, p)
    out = plan.simulate_patch(seed, r, dirs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    ref = ogather.gather(ofield.field(onoise.halfgrid(N, L, seed, k, p)), L, r, hp.cap_directions(32, z_min),
                         "tricubic")
    err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(ref**2))
    assert err <= 1e-12, err
    plan.close()
