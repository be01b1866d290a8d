"""Learned C_l -> P_inf surrogate: a small MLP trained on the linear-programme inversion.

The plain inversion (``spectrum.invert``, Sec. II B) solves a linear programme per
spectrum. The surrogate replaces it by one forward pass of an MLP whose matrix products,
activations, loss and optimiser all run in the library's kernels (``cmbx_mlp_*``): BF16
weights, FP32 accumulation on the matrix cores, FP32 master weights for Adam.

Geometry: a polar cap of half-angle THETA_MAX on a shell of radius R = (r/L) L in a box of
side L = 1. In those units the programme's unknowns sit at k_j R = j pi / (3 sin THETA_MAX),
independent of R, so the network predicts the programme's own unknowns on that fixed grid:

* input (130): log10 of D_l = l(l+1) C_l / 2 pi at 128 log-spaced multipoles in [2, l_max]
  (linear in log l between integer l), shifted by +10; then N / 256 and 2 r / L.
* output (256): y_j = 100 x P_inf(k_j) 4 pi k_j^2 dk / xi_sph(0) for j = 1..256, the
  percentage of xi(0) carried by node j (the programme is homogeneous in C_l, so y does
  not depend on the amplitude); nodes above the box's band limit are zero.

The prediction is accepted only if it reproduces the target correlations inside the cap:
max_i |(A x)_i - b_i| / xi_sph(0) <= tol on the programme's own constraints; otherwise the
plain inversion runs (fallback).
"""
import ctypes
import math
import os
import time

import numpy as np

from . import spectrum, workloads

THETA_MAX = math.radians(30.0)
N_IN, N_OUT, HIDDEN = 130, 256, (512, 512, 512)
L_BOX = 1.0


def kgrid_R():
    """k_j R of the output nodes j = 1..256."""
    return np.arange(1, N_OUT + 1) * math.pi / (3.0 * math.sin(THETA_MAX))


def lmax_of(N, r_over_L):
    return workloads.lmax_for(N, L_BOX, r_over_L)


def features(cl, N, r_over_L):
    cl = np.asarray(cl, dtype=np.float64)
    lmax = cl.size - 1
    l = np.arange(lmax + 1, dtype=np.float64)
    dl = np.zeros_like(cl)
    dl[2:] = l[2:] * (l[2:] + 1) * cl[2:] / (2 * math.pi)
    ls = np.exp(np.linspace(math.log(2.0), math.log(lmax), 128))
    logd = np.log10(np.maximum(dl[2:], 1e-300))
    f = np.interp(np.log(ls), np.log(l[2:]), logd) + 10.0
    return np.concatenate([f, [N / 256.0, 2.0 * r_over_L]]).astype(np.float32)


def label_from_solution(k, p, cl, R):
    """The network target from a programme solution (k, P_inf)."""
    xi0 = spectrum.xi_sph(np.array([0.0]), cl)[0]
    dk = k[1] - k[0]
    y = np.zeros(N_OUT)
    n = min(N_OUT, k.size - 1)
    y[:n] = 100.0 * p[1:n + 1] * 4 * math.pi * k[1:n + 1] ** 2 * dk / xi0
    return y.astype(np.float32)


def table_from_output(y, cl, N, r_over_L):
    """(k, P_inf) table from a network output; nodes beyond the band limit are dropped."""
    R = r_over_L * L_BOX
    dk = math.pi / (3.0 * math.sin(THETA_MAX)) / R
    k_max = math.pi * N / L_BOX
    n = min(N_OUT, int(math.floor(k_max / dk + 1e-9)))
    xi0 = spectrum.xi_sph(np.array([0.0]), cl)[0]
    k = dk * np.arange(n + 1)
    p = np.zeros(n + 1)
    p[1:] = np.maximum(np.asarray(y[:n], dtype=np.float64), 0.0) / 100.0 * xi0 / (4 * math.pi * k[1:] ** 2 * dk)
    return k, p


def cap_residual(k, p, cl, N, r_over_L):
    """max_i |(A x)_i - b_i| / xi_sph(0) on the programme's constraints for this spectrum."""
    lmax = np.asarray(cl).size - 1
    pr = spectrum.lp_problem(cl, r_over_L * L_BOX, THETA_MAX, 1.0 / (0.6 * lmax), math.pi * N / L_BOX)
    x = np.interp(pr["k"], k, p, right=0.0)
    return float(np.max(np.abs(pr["A"] @ x - pr["b"])) / pr["b"][0])


# ---------------------------------------------------------------------------- data
def sample_params(rng):
    N = int(rng.choice([128, 256]))
    r = float(rng.uniform(0.35, 0.45))
    lmax = lmax_of(N, r)
    return dict(N=N, r=r, amp=float(rng.uniform(0.5, 2.0)) * 1e-10, tilt=float(rng.uniform(-0.2, 0.2)),
                period=float(rng.uniform(150.0, 300.0)), phase=float(rng.uniform(0.0, 2 * math.pi)),
                ld=float(rng.uniform(0.4, 0.8)) * lmax)


def cl_of(prm):
    lmax = lmax_of(prm["N"], prm["r"])
    return workloads.shaped_cl(lmax, prm["amp"], prm["tilt"], prm["period"], prm["phase"], prm["ld"])


def plain_inversion(prm, cl=None):
    cl = cl_of(prm) if cl is None else cl
    return spectrum.invert(cl, prm["r"] * L_BOX, THETA_MAX, 1.0 / prm["ld"], N=prm["N"], L=L_BOX)


def _pair(seed):
    rng = np.random.default_rng(seed)
    prm = sample_params(rng)
    cl = cl_of(prm)
    k, p, _ = plain_inversion(prm, cl)
    return features(cl, prm["N"], prm["r"]), label_from_solution(k, p, cl, prm["r"] * L_BOX)


def generate_pairs(n, seed=0, workers=None):
    """n (feature, label) pairs from the plain inversion, seeds seed .. seed + n - 1."""
    seeds = list(range(seed, seed + n))
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    if workers > 1 and n > 8:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            out = list(ex.map(_pair, seeds, chunksize=8))
    else:
        out = [_pair(s) for s in seeds]
    X = np.stack([o[0] for o in out])
    Y = np.stack([o[1] for o in out])
    return X, Y


# ---------------------------------------------------------------------------- network
class MLP:
    """The network on the device; parameters as torch tensors (memory only)."""

    def __init__(self, sizes=(N_IN,) + HIDDEN + (N_OUT,), seed=0, device="cuda"):
        import torch
        from . import cmbx
        self.torch, self.cmbx = torch, cmbx
        self.sizes = tuple(sizes)
        g = np.random.default_rng(seed)
        self.W, self.b, self.Wbf, self.mW, self.vW, self.mb, self.vb = [], [], [], [], [], [], []
        for fi, fo in zip(sizes[:-1], sizes[1:]):
            w = g.normal(0.0, math.sqrt(2.0 / fi), (fi, fo)).astype(np.float32)
            self.W.append(torch.tensor(w, device=device))
            self.b.append(torch.zeros(fo, dtype=torch.float32, device=device))
            self.Wbf.append(torch.empty((fi, fo), dtype=torch.int16, device=device))
            for lst, shape in ((self.mW, (fi, fo)), (self.vW, (fi, fo)), (self.mb, (fo,)), (self.vb, (fo,))):
                lst.append(torch.zeros(shape, dtype=torch.float32, device=device))
        self.step = 0
        self.refresh_bf16()

    def _s(self):
        return self.torch.cuda.current_stream().cuda_stream

    def refresh_bf16(self):
        for w, wb in zip(self.W, self.Wbf):
            self.cmbx._check(self.cmbx.lib().cmbx_bf16_round(w.data_ptr(), wb.data_ptr(), w.numel(), self._s()))

    def forward(self, X):
        """X: (B, 130) float32 CUDA tensor. Returns (out, cache)."""
        torch, L = self.torch, self.cmbx.lib()
        a = X.contiguous()
        cache = []
        nl = len(self.W)
        for li in range(nl):
            fi, fo = self.sizes[li], self.sizes[li + 1]
            B = a.shape[0]
            z = torch.empty((B, fo), dtype=torch.float32, device=a.device)
            y = torch.empty_like(z) if li < nl - 1 else None
            self.cmbx._check(L.cmbx_mlp_gemm(B, fo, fi, a.data_ptr(), fi, 0, self.Wbf[li].data_ptr(), fo, 0, 1,
                                             z.data_ptr(), fo, self.b[li].data_ptr(), 1 if y is not None else 0,
                                             y.data_ptr() if y is not None else None, fo, self._s()))
            cache.append((a, z))
            a = y if y is not None else z
        return a, cache

    def backward(self, cache, dY):
        """Gradients (dW list, db list) for output gradient dY."""
        torch, L = self.torch, self.cmbx.lib()
        nl = len(self.W)
        dWs, dbs = [None] * nl, [None] * nl
        g = dY.contiguous()
        for li in range(nl - 1, -1, -1):
            a, z = cache[li]
            B, fi, fo = a.shape[0], self.sizes[li], self.sizes[li + 1]
            if li < nl - 1:
                dz = torch.empty_like(z)
                self.cmbx._check(L.cmbx_mlp_gelu_backward(z.data_ptr(), g.data_ptr(), dz.data_ptr(), z.numel(),
                                                          self._s()))
            else:
                dz = g
            dW = torch.empty((fi, fo), dtype=torch.float32, device=a.device)
            # dW = a^T dz   (op(A) = a^T: fi x B, op(B) = dz: B x fo)
            self.cmbx._check(L.cmbx_mlp_gemm(fi, fo, B, a.data_ptr(), fi, 1, dz.data_ptr(), fo, 0, 0,
                                             dW.data_ptr(), fo, None, 0, None, fo, self._s()))
            db = torch.empty(fo, dtype=torch.float32, device=a.device)
            self.cmbx._check(L.cmbx_mlp_colsum(dz.data_ptr(), B, fo, db.data_ptr(), self._s()))
            dWs[li], dbs[li] = dW, db
            if li > 0:
                # dA = dz W^T   (op(B) = W^T: W is fi x fo in memory, i.e. transB with ldb = fo)
                ga = torch.empty((B, fi), dtype=torch.float32, device=a.device)
                self.cmbx._check(L.cmbx_mlp_gemm(B, fi, fo, dz.data_ptr(), fo, 0, self.Wbf[li].data_ptr(), fo, 1, 1,
                                                 ga.data_ptr(), fi, None, 0, None, fi, self._s()))
                g = ga
        return dWs, dbs

    def loss_grad(self, out, T, scratch=None):
        torch, L = self.torch, self.cmbx.lib()
        n = out.numel()
        dY = torch.empty_like(out)
        part = torch.empty(int(L.cmbx_mlp_mse_partials(n)), dtype=torch.float32, device=out.device)
        loss = torch.empty(1, dtype=torch.float32, device=out.device)
        self.cmbx._check(L.cmbx_mlp_mse(out.data_ptr(), T.data_ptr(), n, dY.data_ptr(), part.data_ptr(),
                                        loss.data_ptr(), self._s()))
        return loss, dY

    def adam_step(self, dWs, dbs, lr, b1=0.9, b2=0.999, eps=1e-8):
        L = self.cmbx.lib()
        self.step += 1
        for li in range(len(self.W)):
            self.cmbx._check(L.cmbx_mlp_adam(self.W[li].data_ptr(), self.mW[li].data_ptr(), self.vW[li].data_ptr(),
                                             dWs[li].data_ptr(), self.W[li].numel(), lr, b1, b2, eps, self.step,
                                             self.Wbf[li].data_ptr(), self._s()))
            self.cmbx._check(L.cmbx_mlp_adam(self.b[li].data_ptr(), self.mb[li].data_ptr(), self.vb[li].data_ptr(),
                                             dbs[li].data_ptr(), self.b[li].numel(), lr, b1, b2, eps, self.step,
                                             None, self._s()))

    def train(self, X, Y, steps=2000, batch=256, lr=1e-3, seed=0, log_every=0):
        """Minibatch Adam on (X, Y) float32 arrays; returns the list of losses (host floats)."""
        torch = self.torch
        Xd = torch.tensor(X, device="cuda")
        Yd = torch.tensor(Y, device="cuda")
        g = np.random.default_rng(seed)
        losses = []
        for it in range(steps):
            idx = torch.tensor(g.integers(0, X.shape[0], batch), device="cuda")
            xb, yb = Xd[idx].contiguous(), Yd[idx].contiguous()
            out, cache = self.forward(xb)
            loss, dY = self.loss_grad(out, yb)
            dWs, dbs = self.backward(cache, dY)
            step_lr = lr * 0.5 * (1 + math.cos(math.pi * it / steps))
            self.adam_step(dWs, dbs, step_lr)
            if log_every and (it % log_every == 0 or it == steps - 1):
                losses.append((it, float(loss.item())))
        return losses

    def predict(self, X):
        torch = self.torch
        out, _ = self.forward(torch.tensor(np.atleast_2d(X).astype(np.float32), device="cuda"))
        return out.cpu().numpy()

    def state(self):
        return {f"W{i}": w.cpu().numpy() for i, w in enumerate(self.W)} | \
               {f"b{i}": b.cpu().numpy() for i, b in enumerate(self.b)}

    def load_state(self, st):
        for i in range(len(self.W)):
            self.W[i].copy_(self.torch.tensor(st[f"W{i}"]))
            self.b[i].copy_(self.torch.tensor(st[f"b{i}"]))
        self.refresh_bf16()


class Surrogate:
    """C_l -> (k, P_inf) through the network, with the plain inversion as fallback."""

    def __init__(self, mlp, tol=0.01):
        self.mlp, self.tol = mlp, tol
        self.stats = dict(accepted=0, fallback=0)

    def in_domain(self, N, r_over_L):
        return N in (128, 256) and 0.35 <= r_over_L <= 0.45

    def spectrum(self, cl, N, r_over_L, beam=None):
        """Returns (k, P_inf, used_fallback, cap_residual)."""
        if self.in_domain(N, r_over_L):
            y = self.mlp.predict(features(cl, N, r_over_L))[0]
            k, p = table_from_output(y, cl, N, r_over_L)
            res = cap_residual(k, p, cl, N, r_over_L)
            if res <= self.tol:
                self.stats["accepted"] += 1
                return k, p, False, res
        self.stats["fallback"] += 1
        lmax = np.asarray(cl).size - 1
        b = beam if beam is not None else 1.0 / (0.6 * lmax)
        k, p, _ = spectrum.invert(cl, r_over_L * L_BOX, THETA_MAX, b, N=N, L=L_BOX)
        return k, p, True, cap_residual(k, p, cl, N, r_over_L)
