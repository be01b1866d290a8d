"""Host-side pieces of the spectrum surrogate: features, targets and their round trip."""
import math

import numpy as np
import pytest

from paper_2507_15703_amd import spectrum, surrogate, workloads


def _prm(seed):
    return surrogate.sample_params(np.random.default_rng(seed))


def test_features_shape_and_amplitude_shift():
    prm = _prm(3)
    cl = surrogate.cl_of(prm)
    f = surrogate.features(cl, prm["N"], prm["r"])
    assert f.shape == (130,) and np.all(np.isfinite(f))
    f2 = surrogate.features(2.0 * cl, prm["N"], prm["r"])
    assert np.allclose(f2[:128] - f[:128], math.log10(2.0), atol=1e-5)
    assert f[128] == prm["N"] / 256.0 and f[129] == pytest.approx(2 * prm["r"])


def test_target_round_trip_reproduces_programme_solution():
    prm = _prm(5)
    cl = surrogate.cl_of(prm)
    k, p, info = surrogate.plain_inversion(prm, cl)
    y = surrogate.label_from_solution(k, p, cl, prm["r"])
    # the r = 0 constraint holds with equality: the targets sum to 100 % of xi(0)
    assert y.sum() == pytest.approx(100.0, rel=1e-3)
    k2, p2 = surrogate.table_from_output(y, cl, prm["N"], prm["r"])
    assert np.allclose(k2, k[: k2.size], rtol=1e-12)
    assert np.allclose(p2, p[: k2.size], rtol=1e-5, atol=1e-7 * p.max())
    # and the plain solution passes the surrogate's acceptance test
    assert surrogate.cap_residual(k, p, cl, prm["N"], prm["r"]) < 1e-4


def test_targets_do_not_depend_on_amplitude():
    prm = _prm(7)
    cl = surrogate.cl_of(prm)
    k, p, _ = surrogate.plain_inversion(prm, cl)
    k2, p2, _ = surrogate.plain_inversion(prm, 3.0 * cl)
    y1 = surrogate.label_from_solution(k, p, cl, prm["r"])
    y2 = surrogate.label_from_solution(k2, p2, 3.0 * cl, prm["r"])
    assert np.allclose(y1, y2, atol=1e-3)
