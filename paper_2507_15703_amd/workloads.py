"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds input generators only: pixel directions of a polar cap, tabulated
spectra, synthetic angular power spectra and the mixed-size job list of the ensemble
workload. It contains none of the simulator's arithmetic and imports nothing else from
this package, so the HIP path and the CPU oracle can both draw their inputs from it.

Pixelisation: the paper samples the first rings of a HEALPix map (Sec. II D 1); HEALPix is
not used here. A cap of half-angle theta_max is covered by n_ring rings at the mid-points
of equal steps in cos(theta), each with n_phi pixels at phi_j = 2 pi j / n_phi, ordered
ring-major. Pixels of such a grid have equal area.
"""
import math

import numpy as np


def cap_directions(theta_max_deg, n_ring, n_phi):
    """Unit vectors (n_ring * n_phi, 3), float64, of a polar cap, ring-major."""
    ct_max = math.cos(math.radians(theta_max_deg))
    i = np.arange(n_ring, dtype=np.float64)
    cos_t = 1.0 - (i + 0.5) * (1.0 - ct_max) / n_ring
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = 2.0 * np.pi * np.arange(n_phi, dtype=np.float64) / n_phi
    d = np.empty((n_ring, n_phi, 3))
    d[:, :, 0] = sin_t[:, None] * np.cos(phi)[None, :]
    d[:, :, 1] = sin_t[:, None] * np.sin(phi)[None, :]
    d[:, :, 2] = cos_t[:, None]
    return d.reshape(-1, 3)


def random_directions(n, seed):
    """n unit vectors drawn uniformly on the sphere (for edge-case tests)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def powerlaw_cutoff_table(N, L, kc_modes=16.0):
    """P_inf(k) = k^-3 exp(-(k/k_c)^2), k_c = 2 pi kc_modes / L, tabulated on every lattice |k|.

    Nodes k_m = (2 pi / L) sqrt(m), m = 0 .. 3 (N/2)^2; the k = 0 entry is 0.
    """
    two_pi = 6.283185307179586
    k = (two_pi / L) * np.sqrt(np.arange(3 * (N // 2) ** 2 + 1, dtype=np.float64))
    kc = two_pi * kc_modes / L
    p = np.zeros_like(k)
    p[1:] = k[1:] ** -3.0 * np.exp(-((k[1:] / kc) ** 2))
    return k, p


def gaussian_table(L, amp, s, n=4096, kmax_factor=8.0):
    """P_inf(k) = amp exp(-(k s)^2 / 2) on n nodes over [0, kmax_factor / s]."""
    k = np.linspace(0.0, kmax_factor / s, n)
    return k, amp * np.exp(-0.5 * (k * s) ** 2)


def lmax_for(N, L, r):
    """Largest multipole of the synthetic spectra: floor(0.8 pi r N / L)."""
    return int(math.floor(0.8 * math.pi * r * N / L))


def synthetic_cl(lmax, amp=1e-10, ld=None):
    """C_l, l = 0 .. lmax, with l(l+1) C_l / 2 pi = amp (1 + 0.3 cos(pi l / 220)) exp(-(l/ld)^2)
    for l >= 2 and C_0 = C_1 = 0; ld defaults to 0.6 lmax."""
    if ld is None:
        ld = 0.6 * lmax
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    ll = l[2:]
    cl[2:] = amp * (1.0 + 0.3 * np.cos(np.pi * ll / 220.0)) * np.exp(-((ll / ld) ** 2)) * 2.0 * np.pi / (ll * (ll + 1.0))
    return cl


def shaped_cl(lmax, amp, tilt, period, phase, ld):
    """The surrogate's C_l family: l(l+1) C_l / 2 pi = amp (l/100)^tilt
    (1 + 0.3 cos(2 pi l / period + phase)) exp(-(l/ld)^2), l >= 2."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    ll = l[2:]
    dl = amp * (ll / 100.0) ** tilt * (1.0 + 0.3 * np.cos(2.0 * np.pi * ll / period + phase)) * np.exp(-((ll / ld) ** 2))
    cl[2:] = dl * 2.0 * np.pi / (ll * (ll + 1.0))
    return cl


def ensemble_jobs(seed=3):
    """The mixed-size ensemble: 16 x 128^3 + 8 x 256^3 + 4 x 384^3 + 4 x 512^3 boxes.

    Each job: dict(N, seed, r_over_L, theta_deg, amp, n_ring, n_phi). Cap half-angle
    U[10, 40] deg and spectrum amplitude U[0.8, 1.2] are drawn from default_rng(seed);
    n_ring = round(25.6 theta), n_phi = 1024 for theta <= 20 deg else 2048
    (about 256k to 2.1M directions); per-job seeds 3000 + j.
    """
    rng = np.random.default_rng(seed)
    sizes = [128] * 16 + [256] * 8 + [384] * 4 + [512] * 4
    jobs = []
    for j, N in enumerate(sizes):
        theta = float(rng.uniform(10.0, 40.0))
        amp = float(rng.uniform(0.8, 1.2))
        jobs.append(dict(N=N, seed=3000 + j, r_over_L=0.45, theta_deg=theta, amp=amp,
                         n_ring=int(round(25.6 * theta)), n_phi=1024 if theta <= 20.0 else 2048))
    return jobs
