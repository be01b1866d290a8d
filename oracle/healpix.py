"""HEALPix RING pixel centres of a polar cap (test infrastructure only).

Sec. II D 1 evaluates the interpolated box at the sky pixels of a cap centred on the pole,
which are the leading pixels of a HEALPix map stored in RING order. The pixelization is
the published one (K. M. Gorski et al., ApJ 622 (2005) 759, Sec. 4), built here ring by
ring from its definition, for resolution n = Nside (12 n^2 pixels on 4n - 1 rings
i = 1 .. 4n - 1, counted from the north pole):

* north polar rings, i < n: 4 i pixels at z = 1 - i^2 / (3 n^2), longitudes
  phi = (j + 1/2) pi / (2 i), j = 0 .. 4i - 1;
* equatorial rings, n <= i <= 3n: 4 n pixels at z = 4/3 - 2 i / (3 n), longitudes
  phi = (j + 1/2) pi / (2 n) when i + n is even and phi = j pi / (2 n) when it is odd
  (rings alternate between the two offsets; the ring i = n continues the polar pattern);
* south polar rings, i > 3n: the mirror of ring 4n - i, same longitudes, z negated.

RING order runs through the rings from north to south, each in increasing longitude.
Directions are (sin t cos phi, sin t sin phi, z) with sin t = sqrt((1 - z)(1 + z)).

Reading used for the cap (the paper names the cap only by its edge z_min = cos theta_max):
the cap holds every ring whose z is >= z_min; each ring's z is formed as one correctly
rounded FP64 quotient of exact integers, (3n^2 - i^2) / (3n^2) and (4n - 2i) / (3n) (the
south rings negate their mirror's), so that every implementation takes the same decision
at the edge.
"""
import math

import numpy as np


def ring_z(nside, i):
    """z of ring i (1 .. 4n - 1) as the integer quotient described above."""
    n = int(nside)
    if not 1 <= i <= 4 * n - 1:
        raise ValueError("ring index out of range")
    if i < n:
        return float(3 * n * n - i * i) / float(3 * n * n)
    if i <= 3 * n:
        return float(4 * n - 2 * i) / float(3 * n)
    return -ring_z(n, 4 * n - i)


def ring_longitudes(nside, i):
    """Longitudes of ring i in increasing order (FP64)."""
    n = int(nside)
    if i > 3 * n:
        return ring_longitudes(n, 4 * n - i)
    if i < n:
        j = np.arange(4 * i, dtype=np.float64)
        return (j + 0.5) * (math.pi / (2 * i))
    j = np.arange(4 * n, dtype=np.float64)
    shift = 0.5 if (i + n) % 2 == 0 else 0.0
    return (j + shift) * (math.pi / (2 * n))


def rings(nside):
    """[(z, longitudes)] for rings 1 .. 4n - 1, north to south."""
    n = int(nside)
    if n < 1:
        raise ValueError("nside must be >= 1")
    return [(ring_z(n, i), ring_longitudes(n, i)) for i in range(1, 4 * n)]


def directions(z, phi):
    """Unit vectors of pixels at height z and longitudes phi."""
    phi = np.asarray(phi, dtype=np.float64)
    st = math.sqrt((1.0 - z) * (1.0 + z))
    out = np.empty((phi.size, 3))
    out[:, 0] = st * np.cos(phi)
    out[:, 1] = st * np.sin(phi)
    out[:, 2] = z
    return out


def all_pixels(nside):
    """Directions of all 12 n^2 pixels in RING order, shape (12 n^2, 3)."""
    return np.concatenate([directions(z, phi) for z, phi in rings(nside)])


def cap_count(nside, z_min):
    """Number of pixels in the rings with z >= z_min."""
    return sum(phi.size for z, phi in rings(nside) if z >= z_min)


def cap_directions(nside, z_min):
    """Directions of the cap's pixels, the leading cap_count pixels of RING order."""
    parts = [directions(z, phi) for z, phi in rings(nside) if z >= z_min]
    return np.concatenate(parts) if parts else np.zeros((0, 3))
