"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_15703_amd import cmbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(cmbx.LIB_PATH):
        from paper_2507_15703_amd import build
        build.build()
    return cmbx.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "cmbx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmbx_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "cmbx_plan_box" in names and "cmbx_simulate_patch" in names and "cmbx_spectrum_table" in names
    for n in names:
        assert hasattr(L, n), n


def test_version(L):
    assert "gfx950" in cmbx.version()


def _plan(N, Lbox, dt, batch):
    h = ctypes.c_void_p()
    rc = cmbx.lib().cmbx_plan_box(N, Lbox, dt, batch, ctypes.byref(h))
    return rc, h.value


@pytest.mark.parametrize("args,code", [
    ((7, 1.0, cmbx.F32, 1), cmbx.EINVAL),      # odd
    ((4, 1.0, cmbx.F32, 1), cmbx.EINVAL),      # too small
    ((2048, 1.0, cmbx.F32, 1), cmbx.EINVAL),   # too large
    ((64, 0.0, cmbx.F32, 1), cmbx.EINVAL),
    ((64, -1.0, cmbx.F32, 1), cmbx.EINVAL),
    ((64, float("nan"), cmbx.F32, 1), cmbx.EINVAL),
    ((64, float("inf"), cmbx.F32, 1), cmbx.EINVAL),
    ((64, 1.0, 3, 1), cmbx.EINVAL),
    ((64, 1.0, cmbx.F32, 0), cmbx.EINVAL),
    ((80, 1.0, cmbx.F32, 1), cmbx.EUNSUPPORTED),  # 2^4 * 5
    ((36, 1.0, cmbx.F32, 1), cmbx.EUNSUPPORTED),  # 2^2 * 3^2: not compiled
])
def test_plan_box_rejects(L, args, code):
    rc, h = _plan(*args)
    assert rc == code and h is None
    assert cmbx.last_error() != ""


def test_null_arguments(L):
    assert L.cmbx_plan_box(64, 1.0, cmbx.F32, 1, None) == cmbx.EINVAL
    assert L.cmbx_spectrum_table(None, None, None, 2) == cmbx.EINVAL
    assert L.cmbx_simulate_patch(None, 0, 0.4, None, 1, None) == cmbx.EINVAL
    assert L.cmbx_debug_noise(None, 0, None) == cmbx.EINVAL
    assert L.cmbx_debug_field(None, 0, None) == cmbx.EINVAL
    assert L.cmbx_debug_gather(None, None, 0.1, None, 1, None) == cmbx.EINVAL
    assert L.cmbx_debug_footprint(None, 0.1, None, 1, None) == cmbx.EINVAL
    assert L.cmbx_plan_autotune_patch(None, 1, 0.1, None, 1, None, None) == cmbx.EINVAL
    assert L.cmbx_plan_set(None, cmbx.OPT_INTERP, 1) == cmbx.EINVAL
    assert L.cmbx_ensemble_create(None, 0, 0, None) == cmbx.EINVAL
    assert L.cmbx_ensemble_launch(None, None) == cmbx.EINVAL
    assert L.cmbx_ensemble_lanes(None) == cmbx.EINVAL
    assert L.cmbx_plan_destroy(None) == cmbx.OK
    assert L.cmbx_ensemble_destroy(None) == cmbx.OK


def test_valid_plan_without_device_reports_ehip(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    rc, h = _plan(64, 1.0, cmbx.F32, 1)
    assert rc == cmbx.EHIP and h is None
    assert "device" in cmbx.last_error()


def test_noise_tables_match_oracle(L):
    """The library's binary32 Box-Muller tables (host-generated, no device) equal the
    oracle's entry for entry."""
    import ctypes

    from oracle import normal
    buf = (ctypes.c_float * 768)()
    assert L.cmbx_noise_tables(buf, 768) == 768
    got = np.frombuffer(buf, dtype=np.float32)
    ref = np.concatenate([normal.LN_TAB_F, normal.INV_TAB_F, normal.SIN_TAB_F, normal.COS_TAB_F])
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert L.cmbx_noise_tables(buf, 100) == cmbx.EINVAL
    assert L.cmbx_noise_tables(None, 768) == cmbx.EINVAL


def test_footprint_bytes(L):
    """Marks (N planes + N ceil(N/8) row blocks + ceil(N/32) z blocks, padded to 4
    bytes), the lists' header (4 words) and room for one z-list entry per (ix, iy) line
    and one plane-list entry per plane."""
    for N in (8, 12, 48, 512, 1024):
        nb, nzb = (N + 7) // 8, (N + 31) // 32
        assert L.cmbx_footprint_bytes(N) == (N * (1 + nb) + nzb + 3) // 4 * 4 + 16 + 4 * N * N + 4 * N
    assert L.cmbx_footprint_bytes(4) == cmbx.EINVAL
    assert L.cmbx_footprint_bytes(2048) == cmbx.EINVAL


def test_ensemble_rejects_too_many_lanes(L):
    """More than four lanes is refused before anything touches the device (the flags are
    checked before the job list)."""
    h = ctypes.c_void_p()
    rc = L.cmbx_ensemble_create(None, 0, (cmbx.ENS_MAX_LANES + 1) << 8, ctypes.byref(h))
    assert rc == cmbx.EINVAL and "lanes" in cmbx.last_error()
    rc = L.cmbx_ensemble_create(None, 0, cmbx.ENS_MAX_LANES << 8, ctypes.byref(h))
    assert rc == cmbx.EINVAL and "job" in cmbx.last_error()


def test_healpix_cap_count_matches_oracle_host_only():
    # the count path of cmbx_healpix_cap runs on the host and touches no device
    import math
    from oracle import healpix as hp
    from paper_2507_15703_amd import cmbx
    for n in (1, 2, 3, 7, 40, 333):
        for z_min in (2.0, 1.0, 0.999, 2.0 / 3.0, 0.5, 1.0 / 3.0, 0.0, -1.0 / 3.0, -2.0 / 3.0, -0.999, -1.0,
                      math.cos(math.radians(26.85))):
            assert cmbx.healpix_cap_count(n, z_min) == hp.cap_count(n, z_min), (n, z_min)


def test_healpix_cap_errors():
    import ctypes
    from paper_2507_15703_amd import cmbx
    L = cmbx.lib()
    cnt = ctypes.c_int64(-5)
    assert L.cmbx_healpix_cap(0, 0.5, None, 0, ctypes.byref(cnt), None) == cmbx.EINVAL
    assert L.cmbx_healpix_cap((1 << 20) + 1, 0.5, None, 0, ctypes.byref(cnt), None) == cmbx.EINVAL
    assert L.cmbx_healpix_cap(4, float("nan"), None, 0, ctypes.byref(cnt), None) == cmbx.EINVAL
    assert L.cmbx_healpix_cap(4, 0.5, None, 0, None, None) == cmbx.EINVAL
    # too little room: refused before any device work, the count still set
    assert L.cmbx_healpix_cap(4, -1.0, ctypes.c_void_p(256), 191, ctypes.byref(cnt), None) == cmbx.EINVAL
    assert cnt.value == 192
    assert "capacity" in cmbx.last_error()


def test_plan_observer_rejects_non_finite():
    import ctypes
    from paper_2507_15703_amd import cmbx
    L = cmbx.lib()
    assert L.cmbx_plan_observer(None, 0.5, 0.5, 0.5) == cmbx.EINVAL


def test_pixel_covariance_argument_errors():
    # refused before any device work
    from paper_2507_15703_amd import cmbx
    L = cmbx.lib()
    p = 256
    assert L.cmbx_pixel_covariance(None, 4, p, 2, p, None) == cmbx.EINVAL
    assert L.cmbx_pixel_covariance(p, 0, p, 2, p, None) == cmbx.EINVAL
    assert L.cmbx_pixel_covariance(p, 65535 * 16 + 1, p, 2, p, None) == cmbx.EINVAL
    assert L.cmbx_pixel_covariance(p, 4, p, -1, p, None) == cmbx.EINVAL
    assert L.cmbx_pixel_covariance(p, 4, p, (1 << 16) + 1, p, None) == cmbx.EINVAL
    assert "lmax" in cmbx.last_error()
