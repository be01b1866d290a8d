"""Pins of the canonical Box-Muller transform against library functions and statistics."""
import numpy as np
import pytest
import scipy.stats

from oracle import normal

RNG = np.random.default_rng(12345)
WORDS = RNG.integers(0, 2**32, size=400_000, dtype=np.uint64)
EDGE = np.array([0, 1, 2, 3, 2**29 - 1, 2**29, 2**29 + 1, 2**30 - 1, 2**30, 2**30 + 1,
                 2**31 - 1, 2**31, 3 * 2**30, 2**32 - 2, 2**32 - 1], dtype=np.uint64)


def _ulp_err(x, ref):
    return np.abs(x - ref) / np.spacing(np.abs(ref))


def test_log_matches_library():
    a = np.concatenate([WORDS, EDGE])
    got = normal.canonical_log_u1(a)
    ref = np.log((a + np.uint64(1)).astype(np.float64) * 2.0**-32)
    nz = ref != 0
    assert np.all(got[~nz] == 0.0)
    assert np.max(_ulp_err(got[nz], ref[nz])) <= 4


def test_log_exact_powers_of_two():
    # a + 1 = 2^j gives ln u1 = (j - 32) ln 2: the head/tail split must reproduce it.
    for j in range(0, 33):
        a = np.array([2**j - 1], dtype=np.uint64)
        got = float(normal.canonical_log_u1(a)[0])
        assert abs(got - (j - 32) * np.log(2.0)) <= 2 * np.spacing(abs((j - 32) * np.log(2.0)) + 1e-300)


def test_sqrt_matches_library():
    x = np.concatenate([RNG.uniform(0, 45, 200_000), 10.0 ** RNG.uniform(-10, 1.7, 50_000), [1.0, 4.0, 2.0]])
    got = normal.canonical_sqrt(x)
    assert np.max(_ulp_err(got, np.sqrt(x))) <= 4
    assert normal.canonical_sqrt(np.array([0.0, -0.0]))[0] == 0.0


def test_sincos_matches_library():
    b = np.concatenate([WORDS, EDGE])
    s, c = normal.canonical_sincos_2pi(b)
    th = 2.0 * np.pi * (b.astype(np.float64) * 2.0**-32)
    # |error| limited by the rounding of the reference angle (< 8e-16) plus a few ulp.
    assert np.max(np.abs(s - np.sin(th))) < 1.5e-15
    assert np.max(np.abs(c - np.cos(th))) < 1.5e-15
    assert np.max(np.abs(s * s + c * c - 1.0)) < 1e-15


def test_sincos_exact_quadrants():
    s, c = normal.canonical_sincos_2pi(np.array([0, 2**30, 2**31, 3 * 2**30], dtype=np.uint64))
    assert list(s) == [0.0, 1.0, 0.0, -1.0]
    assert list(np.abs(c)) == [1.0, 0.0, 1.0, 0.0]
    assert c[0] == 1.0 and c[2] == -1.0


def test_box_muller_radius_zero():
    g_re, g_im = normal.box_muller(np.array([2**32 - 1], dtype=np.uint64), np.array([12345], dtype=np.uint64))
    assert g_re[0] == 0.0 and g_im[0] == 0.0


def test_normal_distribution():
    a = WORDS
    b = RNG.integers(0, 2**32, size=a.size, dtype=np.uint64)
    g_re, g_im = normal.box_muller(a, b)
    n = a.size
    for g in (g_re, g_im):
        assert abs(g.mean()) < 5 / np.sqrt(n)
        assert abs(g.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(scipy.stats.skew(g)) < 5 * np.sqrt(6 / n)
        assert abs(scipy.stats.kurtosis(g)) < 5 * np.sqrt(24 / n)
        assert scipy.stats.kstest(g, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(g_re, g_im)[0, 1]) < 5 / np.sqrt(n)


def test_box_muller_against_library_form():
    a = WORDS[:100_000]
    b = WORDS[100_000:200_000]
    g_re, g_im = normal.box_muller(a, b)
    u1 = (a + np.uint64(1)).astype(np.float64) * 2.0**-32
    u2 = b.astype(np.float64) * 2.0**-32
    R = np.sqrt(-2.0 * np.log(u1))
    ref_re = R * np.cos(2 * np.pi * u2)
    ref_im = R * np.sin(2 * np.pi * u2)
    assert np.max(np.abs(g_re - ref_re)) < 2e-14
    assert np.max(np.abs(g_im - ref_im)) < 2e-14


# ---------------------------------------------------------------- binary32 variant
def test_f32_log_matches_library():
    a = np.concatenate([WORDS, EDGE])
    got = normal.canonical_log_u1_f32(a)
    assert got.dtype == np.float32
    ref = np.log((a + np.uint64(1)).astype(np.float64) * 2.0**-32)
    # a + 1 keeps its leading 24 bits: u1 changes by a relative 2^-23 at most, i.e. ln u1 by
    # an absolute 2^-23, on top of a few binary32 roundings of the result
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= 4 * 2.0**-24 * np.abs(ref) + 2.0**-23)


def test_f32_sqrt_matches_library():
    x = np.concatenate([RNG.uniform(0, 45, 200_000), 10.0 ** RNG.uniform(-9, 1.6, 50_000)]).astype(np.float32)
    got = normal.canonical_sqrt_f32(x)
    assert got.dtype == np.float32
    ref = np.sqrt(x.astype(np.float64))
    assert np.max(np.abs(got - ref) / ref) < 3 * 2.0**-24


def test_f32_sincos_matches_library():
    b = np.concatenate([WORDS, EDGE])
    s, c = normal.canonical_sincos_2pi_f32(b)
    assert s.dtype == np.float32 and c.dtype == np.float32
    th = 2.0 * np.pi * (b.astype(np.float64) * 2.0**-32)
    assert np.max(np.abs(s - np.sin(th))) < 4e-7
    assert np.max(np.abs(c - np.cos(th))) < 4e-7


def test_f32_pair_close_to_f64_pair_and_normal():
    a, b = WORDS[:200_000], WORDS[200_000:]
    g32 = normal.box_muller_f32(a, b)
    g64 = normal.box_muller(a, b)
    for x32, x64 in zip(g32, g64):
        assert x32.dtype == np.float32
        # only radii below ~5e-4 (u1 within 2^-24 of 1) lose relative accuracy
        assert np.max(np.abs(x32 - x64)) < 1e-3
        assert np.percentile(np.abs(x32 - x64), 99.99) < 2e-6
        assert scipy.stats.kstest(x32.astype(np.float64), "norm").pvalue > 1e-4


def test_f32_tables():
    # each entry is its defining value rounded once to binary32: the identities below hold
    # to the rounding of the entries, and the symmetries of sin and cos exactly
    j = np.arange(128)
    c = 1.0 + j / 128.0
    arg = np.where(j >= normal.FOLD_J, c / 2.0, c)
    ln = normal.LN_TAB_F.astype(np.float64)
    assert np.all(np.abs(np.exp(ln) - arg) <= 2 * 2.0**-24 * arg)
    assert np.all(np.abs(normal.INV_TAB_F.astype(np.float64) * c - 1.0) <= 2.0**-24)
    S, C = normal.SIN_TAB_F.astype(np.float64), normal.COS_TAB_F.astype(np.float64)
    assert np.all(np.abs(S * S + C * C - 1.0) <= 2 * 2.0**-24)
    assert np.array_equal(normal.SIN_TAB_F[:64], normal.COS_TAB_F[63::-1])   # sin x = cos(pi/2 - x)
    assert np.array_equal(normal.SIN_TAB_F[128:], -normal.SIN_TAB_F[:128])   # sin(x + pi) = -sin x
    assert np.array_equal(normal.COS_TAB_F[128:], -normal.COS_TAB_F[:128])
    # fold entries are negative, the others non-negative: ln(c_j / 2) < 0 <= ln c_j
    assert np.all(ln[j >= normal.FOLD_J] < 0) and np.all(ln[j < normal.FOLD_J] >= 0) and ln[0] == 0.0


def test_f32_log_sign_near_one():
    # u1 = 1 gives exactly 0 (a zero radius); every u1 < 1 gives ln u1 < 0, also across the
    # fold entries next to u1 = 1
    a = np.arange(2**32 - 2**18, 2**32, dtype=np.uint64)
    got = normal.canonical_log_u1_f32(a)
    assert got[-1] == 0.0 and np.all(got[:-1] < 0)
    g_re, g_im = normal.box_muller_f32(a[-1:], a[:1])
    assert g_re[0] == 0.0 and g_im[0] == 0.0
