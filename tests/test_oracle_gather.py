"""Pins of the oracle's sphere gather: node exactness, polynomial reproduction, library cross-check."""
import numpy as np
import pytest
import scipy.ndimage

from oracle import gather
from paper_2507_15703_amd import workloads


def test_keys_kernel_textbook_values():
    # Keys (1981), a = -1/2: K(0) = 1, K(1) = K(2) = 0, K(1/2) = 9/16, K(3/2) = -1/16.
    v = gather.keys_kernel([0.0, 1.0, 2.0, 0.5, 1.5, -0.5, 2.5])
    assert list(v) == [1.0, 0.0, 0.0, 0.5625, -0.0625, 0.5625, 0.0]


@pytest.mark.parametrize("interp", [gather.TRILINEAR, gather.TRICUBIC])
def test_exact_at_nodes(interp):
    N, L = 16, 1.0
    rng = np.random.default_rng(1)
    fld = rng.standard_normal((N, N, N))
    # r = m * (L / N) along the axes lands exactly on nodes
    r = 5 * L / N
    dirs = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0]], dtype=float)
    got = gather.gather(fld, L, r, dirs, interp)
    c = N // 2
    ref = [fld[c, c, c + 5], fld[c, c, c - 5], fld[c + 5, c, c], fld[c, c - 5, c]]
    assert np.allclose(got, ref, rtol=0, atol=1e-14)


def test_weights_sum_to_one():
    dirs = workloads.random_directions(500, 2)
    for interp in (gather.TRILINEAR, gather.TRICUBIC):
        _, w = gather.stencil(32, 1.0, 0.37, dirs, interp)
        assert np.allclose(w.sum(axis=2), 1.0, atol=1e-14)


def test_polynomial_reproduction():
    # Trilinear reproduces affine fields; Keys (a = -1/2) reproduces quadratics. Sampled
    # well inside the box so no stencil wraps.
    N, L, r = 32, 1.0, 0.3
    dirs = workloads.random_directions(300, 3)
    j = np.indices((N, N, N)).astype(float)
    p = gather.positions(N, L, r, dirs)
    aff = lambda x, y, z: 0.3 + 1.1 * x - 0.7 * y + 0.2 * z
    quad = lambda x, y, z: 0.1 + x * x - 0.5 * y * z + 0.25 * z * z + 0.3 * x * y - y
    got = gather.gather(aff(*j), L, r, dirs, gather.TRILINEAR)
    assert np.allclose(got, aff(*p.T), rtol=0, atol=1e-12)
    got = gather.gather(quad(*j), L, r, dirs, gather.TRICUBIC)
    assert np.allclose(got, quad(*p.T), rtol=0, atol=1e-10)


def test_trilinear_matches_scipy_map_coordinates():
    N, L, r = 24, 2.0, 0.95
    rng = np.random.default_rng(4)
    fld = rng.standard_normal((N, N, N))
    dirs = workloads.random_directions(1000, 5)
    got = gather.gather(fld, L, r, dirs, gather.TRILINEAR)
    p = gather.positions(N, L, r, dirs)
    ref = scipy.ndimage.map_coordinates(fld, p.T, order=1, mode="grid-wrap")
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


def test_periodic_wrap():
    # r close to L/2 pushes stencils across the box edge; the field is periodic.
    N, L = 16, 1.0
    rng = np.random.default_rng(8)
    fld = rng.standard_normal((N, N, N))
    dirs = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
    got = gather.gather(fld, L, 0.49, dirs, gather.TRICUBIC)
    shifted = np.roll(fld, (-3, -3, -3), axis=(0, 1, 2))
    # same sample expressed in the rolled box: positions move by -3 nodes, no wrap needed
    p = gather.positions(N, L, 0.49, dirs) - 3
    ref = []
    for q in p:
        i0 = np.floor(q).astype(int)
        f = q - i0
        acc = 0.0
        for a in range(-1, 3):
            for b in range(-1, 3):
                for c in range(-1, 3):
                    w = gather.keys_kernel(a - f[0]) * gather.keys_kernel(b - f[1]) * gather.keys_kernel(c - f[2])
                    acc += w * shifted[(i0[0] + a) % N, (i0[1] + b) % N, (i0[2] + c) % N]
        ref.append(acc)
    assert np.allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("interp", [gather.TRILINEAR, gather.TRICUBIC])
def test_observer_offset_is_a_periodic_shift(interp):
    # moving the observer by whole cells samples the field shifted by those cells (the box
    # is periodic); the default observer is the box centre
    N, L, r = 16, 2.0, 0.7
    rng = np.random.default_rng(7)
    fld = rng.standard_normal((N, N, N))
    dirs = workloads.cap_directions(35.0, 6, 24)
    base = gather.gather(fld, L, r, dirs, interp)
    np.testing.assert_array_equal(base, gather.gather(fld, L, r, dirs, interp, observer=(1.0, 1.0, 1.0)))
    k = np.array([3, -2, -5])
    obs = 0.5 * L + k * (L / N)
    got = gather.gather(fld, L, r, dirs, interp, observer=obs)
    ref = gather.gather(np.roll(fld, shift=tuple(-k), axis=(0, 1, 2)), L, r, dirs, interp)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_observer_below_centre_reaches_node():
    # observer lowered by s: the pixel straight up at radius r sits at height L/2 - s + r
    N, L = 16, 1.0
    rng = np.random.default_rng(3)
    fld = rng.standard_normal((N, N, N))
    c = N // 2
    got = gather.gather(fld, L, 7 * L / N, np.array([[0.0, 0.0, 1.0]]), gather.TRICUBIC,
                        observer=(0.5 * L, 0.5 * L, 0.5 * L - 4 * L / N))
    assert abs(got[0] - fld[c, c, c + 3]) <= 1e-14
