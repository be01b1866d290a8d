"""Precision study: FP32 and FP64 maps of the HIP path against the FP64 oracle.

    python tests/precision_study.py --N 1024 --cap 40 --rings 4096 --phi 2048 \
        --out precision_1024.json

One realisation (Philox seed --seed) of the box N^3, L = 1, shell r = 0.45 L, on the
polar cap of half-angle --cap as rings uniform in cos(theta) x equally spaced azimuths,
tricubic interpolation. The 3-D spectrum is the inversion oracle's solution of the
programme (Sec. II B) for the synthetic C_l with l(l+1) C_l / 2 pi =
1e-10 (1 + 0.3 cos(pi l / 220)) exp(-(l / l_d)^2), l_max = floor(0.8 pi r N / L),
l_d = 0.6 l_max, beam 1 / (0.6 l_max), k_max = pi N / L. The same table drives the oracle
and both GPU plans.

Reported: max and RMS of |map - oracle| / rms(oracle) for the FP32 and FP64 plans, and the
recovered (pseudo-)C_l of each map on the cap (ring quadrature of the oracle's harmonic
analysis) against the oracle map's, as band ratios over Delta l = 10 up to l_max
(azimuthal orders m <= n_phi / 2). Prints one progress line per stage and one JSON line.
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

from oracle import field as ofield      # noqa: E402
from oracle import gather as ogather    # noqa: E402
from oracle import inversion as oinv    # noqa: E402
from oracle import maps as omaps        # noqa: E402
from oracle import noise as onoise      # noqa: E402
from paper_2507_15703_amd import workloads  # noqa: E402

R_OVER_L = 0.45


def _log(msg, t0):
    print(f"[precision] {time.time() - t0:7.1f} s  {msg}", flush=True)


def spectrum_input(N, cap_deg):
    """(cl, k, P_inf) of the study: synthetic C_l and the oracle programme's solution."""
    lmax = workloads.lmax_for(N, 1.0, R_OVER_L)
    cl = workloads.synthetic_cl(lmax)
    _, b, k, A, c = oinv.programme(cl, R_OVER_L, math.radians(cap_deg), 1.0 / (0.6 * lmax), math.pi * N)
    _, p = oinv.solve(A, b, c)
    return cl, k, p


def oracle_map(N, seed, k, p, dirs, workers, say, chunk=1 << 20, threads=None):
    """The FP64 oracle's map: noise in `workers` processes (only before this process uses
    the GPU) or `threads` threads, the inverse FFT and the gather on as many threads."""
    h = onoise.halfgrid(N, 1.0, seed, k, p, workers=workers, threads=threads)
    say("oracle half grid")
    fld = ofield.field(h, workers=threads or workers)
    del h
    say("oracle field")
    out = np.empty(dirs.shape[0])
    for i in range(0, dirs.shape[0], chunk):
        out[i:i + chunk] = ogather.gather(fld, 1.0, R_OVER_L, dirs[i:i + chunk], "tricubic", threads=threads)
    say("oracle map")
    return out


def gpu_map(N, dtype, seed, k, p, dirs_dev, reps=3):
    import torch
    from paper_2507_15703_amd import cmbx
    plan = cmbx.Plan(N, 1.0, dtype, interp="tricubic")
    try:
        plan.spectrum_table(k, p)
        out = plan.simulate_patch(seed, R_OVER_L, dirs_dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            plan.simulate_patch(seed, R_OVER_L, dirs_dev, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / reps * 1e3
        return out[0].cpu().numpy().astype(np.float64), ms
    finally:
        plan.close()


def run(N=256, cap_deg=30.0, n_ring=1024, n_phi=1024, seed=1, workers=None, log=True, threads=None):
    """The study's result dict. `workers` (processes) only in a process that has not used
    the GPU yet; inside a test session pass `threads` instead."""
    import torch
    t0 = time.time()
    say = (lambda m: _log(m, t0)) if log else (lambda m: None)
    cl, k, p = spectrum_input(N, cap_deg)
    say(f"spectrum table ({k.size} nodes)")
    dirs = workloads.cap_directions(cap_deg, n_ring, n_phi)
    # the oracle (and its worker processes) runs before this process touches the GPU
    ref = oracle_map(N, seed, k, p, dirs, workers, say, threads=threads)
    dirs_dev = torch.tensor(dirs, device="cuda")
    m32, ms32 = gpu_map(N, "f32", seed, k, p, dirs_dev)
    say(f"gpu f32 map ({ms32:.2f} ms per map)")
    m64, ms64 = gpu_map(N, "f64", seed, k, p, dirs_dev)
    say(f"gpu f64 map ({ms64:.2f} ms per map)")
    del dirs_dev
    rms = math.sqrt(np.mean(ref**2))
    res = {"N": N, "cap_deg": cap_deg, "n_pix": int(dirs.shape[0]), "rings": n_ring, "phi": n_phi, "seed": seed,
           "lmax": cl.size - 1, "ms_per_map": {"f32": round(ms32, 3), "f64": round(ms64, 3)}}
    for name, m in (("f32", m32), ("f64", m64)):
        d = np.abs(m - ref) / rms
        res[f"max_rel_{name}"] = float(d.max())
        res[f"rms_rel_{name}"] = float(math.sqrt(np.mean(d**2)))
    ct_max = math.cos(math.radians(cap_deg))
    cos_t = 1.0 - (np.arange(n_ring) + 0.5) * (1.0 - ct_max) / n_ring
    d_omega = (1.0 - ct_max) / n_ring * 2 * math.pi / n_phi
    lmax = cl.size - 1
    alm = omaps.ring_alm(np.stack([ref, m32, m64]), cos_t, n_phi, lmax, d_omega)
    pcl = omaps.pseudo_cl(alm)
    say("recovered C_l")
    for i, name in ((1, "f32"), (2, "f64")):
        br = omaps.band_ratio(pcl[i], pcl[0])
        res[f"cl_band_max_{name}"] = float(np.max(np.abs(br)))
        res[f"cl_band_median_{name}"] = float(np.median(np.abs(br)))
    exp = oinv.cap_pseudo_cl(lambda th: oinv.xi_sph(th, cl), math.radians(cap_deg), lmax)
    br = omaps.band_ratio(pcl[0], exp)
    res["oracle_vs_expected_band_median"] = float(np.median(np.abs(br)))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--cap", type=float, default=40.0)
    ap.add_argument("--rings", type=int, default=4096)
    ap.add_argument("--phi", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run(a.N, a.cap, a.rings, a.phi, a.seed, a.workers)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
