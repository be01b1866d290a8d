"""The paper's covariance test of simulated maps (Sec. III B), with the linear algebra on
the device.

Maps made from a power spectrum are Gaussian with zero mean, so they are right if their
pixel covariance is Gamma_ij = sum_l (2l + 1) C_l P_l(n_i . n_j) / (4 pi) (eq. harmonics).
With Gamma + s^2 I = L L^T, the vector x = L^-1 (m + s w) of a map m plus white noise w of
unit variance should hold independent unit normals; the Kolmogorov-Smirnov statistic of
all entries of x against N(0, 1) decides. Gamma is ill-conditioned, so the paper adds
noise at increasing levels s and reports the smallest level that passes.

Device steps: cmbx_pixel_covariance, cmbx_cholesky (with the shift s^2), cmbx_whiten. The
white noise w is drawn on the host (numpy default_rng(seed), the same unit draws for every
level) and the KS test runs on the host (scipy). Noise levels are fractions of the map
rms sqrt(Gamma_00).
"""
import numpy as np
import scipy.stats

from . import cmbx


def ks_sweep(maps, dirs, cl, noise_fracs, seed=0, alpha=0.05):
    """KS results for every noise level: list of dict(noise_frac, s, D, p, passed).

    maps: (n_maps, n_pix) float64 CUDA tensor (left unchanged); dirs: (n_pix, 3) float64
    CUDA tensor of the pixel directions; cl: C_l for l = 0 .. lmax (host or device)."""
    import torch
    n_maps, n = maps.shape
    gamma0 = cmbx.pixel_covariance(dirs, cl)
    g00 = float(gamma0[0, 0].item())
    w = torch.tensor(np.random.default_rng(seed).standard_normal((n_maps, n)), dtype=torch.float64,
                     device=maps.device)
    out = []
    for frac in noise_fracs:
        s = float(frac) * np.sqrt(g00)
        L = gamma0.clone()
        info = cmbx.cholesky(L, shift=s * s)
        x = maps + s * w
        cmbx.whiten(L, x)
        col = int(info.item())
        if col != 0:
            out.append(dict(noise_frac=float(frac), s=s, D=float("nan"), p=0.0, passed=False, not_pd_at=col))
            continue
        r = scipy.stats.kstest(x.cpu().numpy().ravel(), "norm")
        out.append(dict(noise_frac=float(frac), s=s, D=float(r.statistic), p=float(r.pvalue),
                        passed=bool(r.pvalue > alpha)))
    return out


def noise_to_pass(results):
    """The smallest noise fraction whose KS test passed (None if none did)."""
    ok = [r["noise_frac"] for r in results if r["passed"]]
    return min(ok) if ok else None
