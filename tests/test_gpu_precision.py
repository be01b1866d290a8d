"""Per-pixel error and recovered C_l of the FP32 and FP64 plans against the FP64 oracle on
the 256^3 single-realisation workload: r = 0.45 L, 30-degree cap as 1024 rings x 1024
azimuths, tricubic, Philox seed 1, 3-D spectrum from the programme for the synthetic C_l
(the study in ``precision_study.py`` at this size)."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_precision_256_lp_spectrum():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import precision_study
    res = precision_study.run(N=256, cap_deg=30.0, n_ring=1024, n_phi=1024, seed=1)
    print(res, flush=True)
    assert res["max_rel_f32"] <= 1e-5
    assert res["max_rel_f64"] <= 1e-12
    # the recovered C_l of the maps follow the oracle map's in every Delta l = 10 band
    assert res["cl_band_max_f32"] <= 1e-5
    assert res["cl_band_max_f64"] <= 1e-12
