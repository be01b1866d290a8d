"""Pins of the FP64 MLP oracle: bfloat16 rounding against torch, gradients against finite
differences, GELU derivative, one Adam step in closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100_000).astype(np.float32) * 10.0 ** rng.uniform(-6, 6, 100_000).astype(np.float32),
                        # exact ties between two bfloat16 neighbours
                        (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gelu_grad_finite_difference():
    x = np.linspace(-6, 6, 121)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([50.0]))[0] == 50.0


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    sizes = (5, 7, 6, 3)
    Ws = [rng.standard_normal((a, b)) * 0.7 for a, b in zip(sizes[:-1], sizes[1:])]
    bs = [rng.standard_normal(b) * 0.1 for b in sizes[1:]]
    X = rng.standard_normal((4, sizes[0]))
    T = rng.standard_normal((4, sizes[-1]))

    def loss(Ws_, bs_):
        out, _ = mlp.forward(X, Ws_, bs_, round_bf16=False)
        return mlp.mse(out, T)[0]

    out, cache = mlp.forward(X, Ws, bs, round_bf16=False)
    _, dY = mlp.mse(out, T)
    dWs, dbs = mlp.backward(cache, Ws, dY, round_bf16=False)
    h = 1e-6
    for li in range(len(Ws)):
        for idx in [(0, 0), (1, 2), (Ws[li].shape[0] - 1, Ws[li].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[li][idx] += h
            Wm[li][idx] -= h
            fd = (loss(Wp, bs) - loss(Wm, bs)) / (2 * h)
            assert dWs[li][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[li][0] += h
        bm[li][0] -= h
        assert dbs[li][0] == pytest.approx((loss(Ws, bp) - loss(Ws, bm)) / (2 * h), rel=1e-5, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    # after one step from zero moments the update is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    w, m, v = mlp.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
