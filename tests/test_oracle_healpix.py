"""Pins of the HEALPix cap oracle against properties the pixelization fixes.

Sec. II D 1 samples the cap centred on the pole: the leading pixels of a RING-ordered
HEALPix map. The pins are the twelve base pixels of Nside = 1, the pixel count per ring
and in total, equal pixel areas (the area north of each ring centre equals the area of
the pixels before it plus half its own), the continuity of the polar and equatorial
longitude patterns and the half-pixel offset between neighbouring equatorial rings,
mirror symmetry about the equator, and the cap as a prefix of RING order.
"""
import math

import numpy as np
import pytest

from oracle import healpix as hp


def test_base_pixels_nside1():
    # the 12 base pixels: 4 around z = 2/3 at 45 + 90k degrees, 4 on the equator at 90k
    # degrees, 4 around z = -2/3 at 45 + 90k degrees
    d = hp.all_pixels(1)
    assert d.shape == (12, 3)
    s = math.sqrt(5.0) / 3.0
    expect = []
    for z, offset in ((2.0 / 3.0, 45.0), (0.0, 0.0), (-2.0 / 3.0, 45.0)):
        st = s if z else 1.0
        for k in range(4):
            a = math.radians(offset + 90.0 * k)
            expect.append((st * math.cos(a), st * math.sin(a), z))
    np.testing.assert_allclose(d, np.array(expect), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16])
def test_ring_counts(n):
    r = hp.rings(n)
    assert len(r) == 4 * n - 1
    counts = [phi.size for _, phi in r]
    for i, c in enumerate(counts, start=1):
        k = min(i, n, 4 * n - i)
        assert c == 4 * k
    assert sum(counts) == 12 * n * n
    # pixels north of the polar belt: sum of 4i over i < n
    assert sum(counts[: n - 1]) == 2 * n * (n - 1)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 32])
def test_equal_areas(n):
    # every pixel has area 4 pi / (12 n^2); ring centres sit where the cap above them
    # holds the pixels of the rings before plus half the ring's own
    omega = 4.0 * math.pi / (12 * n * n)
    before = 0
    for z, phi in hp.rings(n):
        area = 2.0 * math.pi * (1.0 - z)
        assert area == pytest.approx(omega * (before + phi.size / 2.0), rel=1e-13, abs=1e-13)
        before += phi.size


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_longitude_patterns(n):
    r = hp.rings(n)
    for z, phi in r:
        step = 2.0 * math.pi / phi.size
        np.testing.assert_allclose(np.diff(phi), step, rtol=1e-13)
        assert 0.0 <= phi[0] < step and phi[-1] < 2.0 * math.pi
    # polar rings start half a pixel from phi = 0; ring n continues that pattern
    for i in range(1, n + 1):
        phi = r[i - 1][1]
        assert phi[0] == pytest.approx(0.5 * 2.0 * math.pi / phi.size, rel=1e-14)
    # neighbouring equatorial rings are offset by half a pixel
    for i in range(n, 3 * n):
        a, b = r[i - 1][1], r[i][1]
        assert abs(a[0] - b[0]) == pytest.approx(math.pi / (4 * n), rel=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 8])
def test_mirror_symmetry(n):
    r = hp.rings(n)
    for i in range(1, 4 * n):
        z, phi = r[i - 1]
        zm, phim = r[4 * n - i - 1]
        assert z == -zm
        np.testing.assert_array_equal(phi, phim)
    d = hp.all_pixels(n)
    np.testing.assert_allclose(d.sum(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 5, 16])
def test_cap_is_ring_prefix(n):
    d = hp.all_pixels(n)
    for zmin in (1.5, 1.0, 0.95, 2.0 / 3.0, 0.3, 0.0, -0.5, -1.0, -2.0):
        c = hp.cap_count(n, zmin)
        cap = hp.cap_directions(n, zmin)
        assert cap.shape == (c, 3)
        np.testing.assert_array_equal(cap, d[:c])
        if c:
            assert cap[:, 2].min() >= zmin
        if c < d.shape[0]:
            assert d[c, 2] < zmin
    # the polar zone (rings 1 .. n, down to z = 2/3) holds 2 n (n + 1) pixels
    assert hp.cap_count(n, 2.0 / 3.0) == 2 * n * (n + 1)
    assert hp.cap_count(n, -1.0) == 12 * n * n
    assert hp.cap_count(n, 1.0 + 1e-12) == 0
