"""FP64 forward and backward of the spectrum surrogate MLP (test infrastructure only).

The network is a stack of affine layers, GELU(x) = x Phi(x) between them and none after the
last, trained on the mean squared error with Adam (Kingma & Ba, ICLR 2015). To compare with
the matrix-core kernels bit-for-bit in their inputs, every GEMM operand is rounded to
bfloat16 (round to nearest even) before an FP64 product, as the kernels round their FP32
operands before the FP32-accumulating matrix instruction.
"""
import math

import numpy as np
from scipy.special import erf


def bf16(x):
    """Round to bfloat16 (nearest even) through binary32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(X, Ws, bs, round_bf16=True):
    """Outputs and the per-layer (input, pre-activation) pairs."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(zip(Ws, bs)):
        z = r(a) @ r(W) + b
        cache.append((a, z))
        a = gelu(z) if li < len(Ws) - 1 else z
    return a, cache


def mse(Y, T):
    d = np.asarray(Y, dtype=np.float64) - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(cache, Ws, dY, round_bf16=True):
    """Gradients (dWs, dbs) of the loss whose output gradient is dY."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    dWs, dbs = [None] * len(Ws), [None] * len(Ws)
    g = np.asarray(dY, dtype=np.float64)
    for li in range(len(Ws) - 1, -1, -1):
        a, z = cache[li]
        dz = g if li == len(Ws) - 1 else g * gelu_grad(z)
        dWs[li] = r(a).T @ r(dz)
        dbs[li] = dz.sum(axis=0)
        if li > 0:
            g = r(dz) @ r(Ws[li]).T
    return dWs, dbs


def adam(w, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1**step)) / (np.sqrt(v / (1 - b2**step)) + eps)
    return w, m, v
