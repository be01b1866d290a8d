"""What the trained spectrum surrogate gains over the plain inversion, judged by the oracle.

Loads the shipped BF16 weights (trained on the GPU by the library's MLP kernels on pairs
from the plain inversion) and runs ``surrogate_study`` on 16 held-out spectra at 256^3,
r = 0.45 L, 30-degree cap: the share the surrogate answers itself, the oracle's in-cap
correlations and expected cap pseudo-C_l of those answers against the target, the
mean recovered C_l of 128 same-seed FP32 maps per spectrum for two of them against the
plain inversion's maps, and spectra/s against the programme.
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_surrogate_gain_over_plain_inversion():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import surrogate_study
    res = surrogate_study.run(n=16, n_maps=2, seeds=128)
    print(res, flush=True)
    assert res["accepted"] >= 12
    # the answers the surrogate keeps: in-cap correlations within 0.2 % of xi(0) and the
    # expected pseudo-C_l within 1 % of the target's in every Delta l = 10 band
    assert res["corr_err_max"] <= 0.002
    assert res["expected_band_max"] <= 0.01
    # maps from the surrogate's spectrum recover the plain inversion's C_l (same seeds, mean
    # of 128 maps): every band within 1 % up to three standard errors of the paired means
    assert res["recovered_ratio_max_beyond_3sigma"] <= 0.01
    assert res["speedup"] >= 20
