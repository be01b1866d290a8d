"""Parity with the FP64 oracle at the sizes the benchmark and the studies actually run.

* The benchmark's launch configuration: the four 512^3 FP32 boxes of the mixed-size
  ensemble, each with the programme's spectrum for its cap (Sec. II B), tricubic, maps
  pruned to their footprint, fixed directions, tiles tuned on each map's pixels, run as
  one chained ensemble on four lanes; every pixel of every map against the oracle, on two
  replays.
* 384^3 (radix-3 transform lengths at size), FP32 and FP64, every pixel.
* The flat-box methods at the benchmark's size (N = 512, M = 32, h = 14): the 2-D (hybrid)
  method and the 3-D method on the flat box, every pixel of a HEALPix cap.
* The precision study at 1024^3 (40-degree cap, 4096 x 2048 pixels): FP32 and FP64 plans
  against one FP64 oracle map, per pixel and per recovered-C_l band.

Bar: max|gpu - oracle| / rms(oracle) <= 1e-5 (FP32), <= 1e-12 (FP64). The oracle takes
the same spectrum table as the plans, made by the oracle's own programme solver, and runs
on threads of this process (it must not fork once the GPU is in use).
"""
import math
import os
import time

import numpy as np
import pytest

from oracle import field as ofield
from oracle import gather as ogather
from oracle import inversion as oinv
from oracle import noise as onoise
from paper_2507_15703_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def cmbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_15703_amd import cmbx as c
    c.lib()
    return c


def _say(msg):
    print(f"[at-size] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def _rel(gpu, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(np.asarray(gpu, dtype=np.float64) - ref)) / np.sqrt(np.mean(ref**2)))


def _job_table(N, r, theta_deg, amp):
    """The job's P_inf table from the oracle's programme: the synthetic C_l family scaled by
    amp, l_max = floor(0.8 pi r N), beam 1 / (0.6 l_max), cap theta, k_max = pi N (L = 1)."""
    lmax = workloads.lmax_for(N, 1.0, r)
    cl = amp * workloads.synthetic_cl(lmax)
    _, b, k, A, c = oinv.programme(cl, r, math.radians(theta_deg), 1.0 / (0.6 * lmax), math.pi * N)
    _, p = oinv.solve(A, b, c)
    return k, p


def _oracle_map(N, seed, k, p, r, dirs, interp):
    h = onoise.halfgrid(N, 1.0, seed, k, p, threads=THREADS)
    fld = ofield.field(h, workers=THREADS)
    del h
    return ogather.gather(fld, 1.0, r, dirs, interp, threads=THREADS)


def test_bench_ensemble_512_every_pixel(cmbx):
    """The 4 x 512^3 FP32 benchmark ensemble (chained, four lanes, LP spectra, pruned,
    patch-tuned tiles, fixed directions: footprints made once and the gathers in pixel
    order): every pixel of every map within 1e-5 of the FP64 oracle."""
    meta = [j for j in workloads.ensemble_jobs() if j["N"] == 512]
    assert len(meta) == 4
    jobs, dirs_np, tables = [], [], []
    for j in meta:
        r = j["r_over_L"]
        k, p = _job_table(512, r, j["theta_deg"], j["amp"])
        tables.append((k, p))
        plan = cmbx.Plan(512, 1.0, "f32", batch=1, interp="tricubic")
        plan.spectrum_table(k, p)
        plan.set_fixed_dirs(True)
        d_np = workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"])
        dirs_np.append(d_np)
        dirs = torch.tensor(d_np, device="cuda")
        plan.autotune(reps=3, r=r, dirs=dirs)
        out = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        jobs.append(dict(plan=plan, seed=j["seed"], r=r, dirs=dirs, out=out))
    _say("plans ready")
    ens = cmbx.Ensemble([dict(j) for j in jobs], mode="chained", lanes=4)
    assert ens.lanes == 4 and ens.modes == ["chained"]
    got = []
    for rep in range(2):
        for j in jobs:
            j["out"].fill_(float("nan"))
        ens.launch()
        torch.cuda.synchronize()
        got.append([j["out"].cpu().numpy()[0].copy() for j in jobs])
    ens.close()
    for j in jobs:
        j["plan"].close()
    _say("ensemble maps done")
    for i, (j, (k, p)) in enumerate(zip(jobs, tables)):
        ref = _oracle_map(512, j["seed"], k, p, j["r"], dirs_np[i], "tricubic")
        for rep in range(2):
            err = _rel(got[rep][i], ref)
            _say(f"job {i} replay {rep}: {dirs_np[i].shape[0]} px, max|d|/rms = {err:.3e}")
            assert np.all(np.isfinite(got[rep][i])) and err <= 1e-5, (i, rep, err)


@pytest.mark.parametrize("dt,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_map_384_every_pixel(cmbx, dt, tol):
    """384^3 (x and y transforms of length 384 = 3 * 2^7, z of 192), the first 384^3 job of
    the ensemble: its cap, spectrum and seed, tricubic, every pixel against the oracle."""
    j = next(j for j in workloads.ensemble_jobs() if j["N"] == 384)
    r = j["r_over_L"]
    k, p = _job_table(384, r, j["theta_deg"], j["amp"])
    d_np = workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"])
    plan = cmbx.Plan(384, 1.0, dt, interp="tricubic")
    plan.spectrum_table(k, p)
    out = plan.simulate_patch(j["seed"], r, torch.tensor(d_np, device="cuda"))
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    plan.close()
    ref = _oracle_map(384, j["seed"], k, p, r, d_np, "tricubic")
    err = _rel(got, ref)
    _say(f"384^3 {dt}: {d_np.shape[0]} px, max|d|/rms = {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("method", ["hybrid", "flat"])
def test_slab_methods_at_the_benchmark_size(cmbx, method):
    """The flat-box methods as the benchmark times them: beam b = 0.01 rad, 10-degree cap on
    the unit sphere, the Sec. II C box (N = 512, M = 32, dp = 0.0017), h = 14 layers for the
    2-D method, the oracle programme's P_inf, FP32, tricubic, every pixel of the HEALPix cap
    at nside 64 against the FP64 oracle (oracle.slab), two realisations."""
    from oracle import healpix as ohp
    from oracle import slab as oslab
    b, theta = 0.01, math.radians(10.0)
    z_min = math.cos(theta)
    N, M, dp = oslab.box_size(b, theta)
    assert (N, M) == (512, 32)
    h = min(M, int(math.ceil((1.0 - z_min) / dp)) + 5)
    cl = workloads.synthetic_cl(int(math.ceil(5.0 / b)), ld=1.0 / b)
    _, bb, k, A, c = oinv.programme(cl, 1.0, theta, b, math.pi / dp)
    _, p = oinv.solve(A, bb, c)
    d_np = ohp.cap_directions(64, z_min)
    s = cmbx.Slab(method, N, M, dp, h=h, dtype="f32", batch=2, interp="tricubic")
    s.spectrum(k, p)
    obs = s.observer_for_cap(1.0, z_min)
    s.set_observer(obs)
    got = s.simulate(77, 1.0, torch.tensor(d_np, device="cuda")).cpu().numpy()
    s.close()
    for i in range(2):
        if method == "hybrid":
            lay = oslab.hybrid_layers(oslab.hybrid_columns(N, M, h, dp, 77 + i, k, p))
        else:
            lay = oslab.flat_layers(oslab.flat_halfgrid(N, M, dp, 77 + i, k, p))
        ref = oslab.gather_layers(lay, dp, 1.0, d_np, "tricubic", obs, periodic_z=method == "flat")
        assert np.all(np.isfinite(ref))
        err = _rel(got[i], ref)
        _say(f"{method} N={N} M={M} h={h}: {d_np.shape[0]} px, realisation {i}, max|d|/rms = {err:.3e}")
        assert err <= 1e-5


@pytest.mark.timeout(900)
def test_precision_study_1024(cmbx):
    """Config 4: one 1024^3 realisation (seed 4), r = 0.45 L, 40-degree cap as 4096 rings x
    2048 azimuths (8.4M pixels), tricubic, spectrum from the programme; the FP32 and FP64
    plans against the FP64 oracle per pixel and per Delta l = 10 band of the recovered C_l."""
    import precision_study
    res = precision_study.run(N=1024, cap_deg=40.0, n_ring=4096, n_phi=2048, seed=4, threads=THREADS)
    print("PRECISION_1024 " + __import__("json").dumps(res), flush=True)
    assert res["n_pix"] == 4096 * 2048
    assert res["max_rel_f32"] <= 1e-5
    assert res["max_rel_f64"] <= 1e-12
    assert res["cl_band_max_f32"] <= 1e-5
    assert res["cl_band_max_f64"] <= 1e-12
