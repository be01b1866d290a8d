"""The paper's decisive validation (Sec. III B) on this build's maps: the added-noise sweep.

    python tests/covariance_study.py --nside 32 --cap 20 --beam-deg 1.72 --maps 1000 [--m-factor 4]

On the unit sphere: C_l of the synthetic family smoothed by a Gaussian beam b (eq. cl,
l(l+1) C_l / 2 pi = 1e-10 (1 + 0.3 cos(pi l / 220)) exp(-(b l)^2), l <= 5 / b), the
programme's P_inf for the cap (Sec. II B, beam b, the host inversion), a box sized by the
rule of Sec. II C (cmbx_box_size) and the maps of the 2-D (hybrid) method on h layers centred
on the cap (Sec. II D 2) -- and, for comparison, of the 3-D method on the whole flat box --
at the pixels of the HEALPix cap of resolution nside (RING order, made on the device).
For every noise level (fractions of the map rms) the maps plus white noise are whitened by
the Cholesky factor of Gamma + s^2 I on the device and KS-tested on the host
(``paper_2507_15703_amd.covtest``). Control: maps drawn exactly from Gamma (on the host,
Cholesky of Gamma plus 1e-12 of its diagonal) must pass at the smallest level.

The box is periodic along z with period M dp. The rule's M (twice the cap's depth) puts
the first periodic images of a pixel within the cap's widest chord, so correlations that
reach that far add to the variance: --m-factor multiplies M (the rule's N is kept). The
expected variance of the box's field, sum P_box over the lattice (oracle ``p_box_flat``),
is printed against xi(0) for each M as the prediction the maps' rms is checked against.

Prints one line per level and method, then one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LEVELS = [0.0, 1e-4, 3e-4, 1e-3, 2e-3, 5e-3, 1e-2, 2e-2, 5e-2, 0.1]


def lattice_variance(N, M, dp, k, p):
    """sum of P_box over the N x N x M lattice (eq. finalpbox): the field's variance."""
    from oracle import slab as oslab
    P = oslab.p_box_flat(N, M, dp, k, p)                 # [s][fz], fz = 0 .. M/2
    f = np.arange(-N // 2, N // 2)
    cnt = np.bincount((f[:, None] ** 2 + f[None, :] ** 2).ravel(), minlength=P.shape[0])
    wz = np.full(M // 2 + 1, 2.0)
    wz[0] = wz[-1] = 1.0
    return float(np.sum(cnt[:, None] * P[: cnt.size] * wz[None, :]))


def run(nside=32, cap_deg=20.0, beam_deg=1.72, n_maps=1000, size_factor=1.0, seed=0, levels=LEVELS, log=True,
        m_factor=1):
    import torch

    from paper_2507_15703_amd import cmbx, covtest, spectrum, workloads

    t0 = time.time()

    def say(msg):
        if log:
            print(f"[covariance] {time.time() - t0:7.1f} s  {msg}", flush=True)

    b = math.radians(beam_deg)
    theta = math.radians(cap_deg)
    z_min = math.cos(theta)
    lmax = int(math.ceil(5.0 / b))
    cl = workloads.synthetic_cl(lmax, ld=1.0 / b)
    N, M, dp = cmbx.box_size(b, theta, size_factor)
    M *= int(m_factor)
    # layers: the cap's height plus the tricubic stencil's two nodes each side
    h = min(M, int(math.ceil((1.0 - z_min) / dp)) + 5)
    k, p, info = spectrum.invert(cl, 1.0, theta, b, k_max=math.pi / dp)
    xi0_sph = float(spectrum.xi_sph(np.zeros(1), cl)[0])
    var_box = lattice_variance(N, M, dp, k, p)
    say(f"box N={N} M={M} h={h} dp={dp:.5g}; programme {info['n_r']}x{info['n_k']}, largest excess "
        f"{info['max_rel_excess']:.4f} of xi(0); lattice variance / xi(0) = {var_box / xi0_sph:.4f}")
    dirs = cmbx.healpix_cap(nside, z_min)
    n_pix = dirs.shape[0]
    res = {"nside": nside, "cap_deg": cap_deg, "beam_deg": beam_deg, "n_pix": n_pix, "n_maps": n_maps,
           "N": N, "M": M, "m_factor": int(m_factor), "h": h, "dp": dp, "lmax": lmax, "levels": list(levels),
           "lattice_var_over_xi0": var_box / xi0_sph, "programme_max_excess": info["max_rel_excess"]}
    batch = 50
    for method in ("hybrid", "flat"):
        slab = cmbx.Slab(method, N, M, dp, h=h, dtype="f32", batch=batch, interp="tricubic")
        slab.spectrum(k, p)
        slab.set_observer(slab.observer_for_cap(1.0, z_min))
        maps = torch.empty((n_maps, n_pix), dtype=torch.float64, device="cuda")
        for s0 in range(0, n_maps, batch):
            m = slab.simulate(seed + s0, 1.0, dirs)
            maps[s0:s0 + batch] = m[: min(batch, n_maps - s0)].double()
        torch.cuda.synchronize()
        slab.close()
        assert bool(torch.isfinite(maps).all()), "a pixel's stencil left the layers"
        rms = float(maps.pow(2).mean().sqrt().item())
        xi0 = float(cmbx.pixel_covariance(dirs[:1], cl)[0, 0].item())
        say(f"{method}: {n_maps} maps, rms {rms:.4g} vs sqrt(xi(0)) {math.sqrt(xi0):.4g}")
        sweep = covtest.ks_sweep(maps, dirs, cl, levels, seed=seed + 1)
        for r in sweep:
            say(f"{method}: noise {100 * r['noise_frac']:7.3f} %  D = {r['D']:.5f}  p = {r['p']:.3g}")
        res[method] = {"rms_over_sqrt_xi0": rms / math.sqrt(xi0), "D": [r["D"] for r in sweep],
                       "p": [r["p"] for r in sweep], "noise_to_pass": covtest.noise_to_pass(sweep)}
        del maps
    # control: exact draws from Gamma
    G = cmbx.pixel_covariance(dirs, cl).cpu().numpy()
    Lc = np.linalg.cholesky(G + 1e-12 * G[0, 0] * np.eye(n_pix))
    z = np.random.default_rng(seed + 2).standard_normal((n_maps, n_pix))
    exact = torch.tensor(z @ Lc.T, device="cuda")
    sweep = covtest.ks_sweep(exact, dirs, cl, levels[:3], seed=seed + 3)
    for r in sweep:
        say(f"exact draws: noise {100 * r['noise_frac']:7.3f} %  D = {r['D']:.5f}  p = {r['p']:.3g}")
    res["exact_draws"] = {"D": [r["D"] for r in sweep], "p": [r["p"] for r in sweep]}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nside", type=int, default=32)
    ap.add_argument("--cap", type=float, default=20.0)
    ap.add_argument("--beam-deg", type=float, default=1.72)
    ap.add_argument("--maps", type=int, default=1000)
    ap.add_argument("--size-factor", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--m-factor", type=int, default=1)
    a = ap.parse_args()
    res = run(a.nside, a.cap, a.beam_deg, a.maps, a.size_factor, a.seed, m_factor=a.m_factor)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
