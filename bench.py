#!/usr/bin/env python3
"""Throughput of the partial-sky box simulator on one MI355X.

Workload: the 512^3 part of the mixed-size ensemble -- four FP32 boxes of side L = 1,
each with its own seed, shell radius r = 0.45 L, a polar cap of half-angle drawn
uniformly in [10, 40] deg (n_ring = round(25.6 theta) rings x 1024 or 2048 pixels) and
tricubic sampling. Each box's P(k) is the programme's solution (host FP64 inversion) for
the synthetic C_l family scaled by the job's amplitude, on the job's cap; it ends at the
box's band limit pi N / L, so the modes beyond it (about half) have zero weight and are
not drawn. One step = one pass of the whole hot path (noise + inverse 3-D FFT +
sphere gather) over the four boxes, i.e. four maps. The batched path replays the four
independent kernel chains as a HIP-graph ensemble (graphs on up to four streams, as the
ensemble's auto mode finds fastest); the plain path runs the same jobs one after another
through cmbx_simulate_patch on one stream. Every plan keeps its directions fixed
(CMBX_OPT_FIXED_DIRS: the paper's batches are many maps of one cap, so each map
footprint is made once, in both paths). Inputs (directions, spectrum tables) are
resident in device memory before timing starts.

Beside the headline line: alternating blocks of batched and plain steps (median and
spread), per-kernel times with their algorithmic bytes, the noise + x pass's ALU
roofline, the 2-D (hybrid) Fourier method and the 3-D method on a flat box of the same
N x N x M, the covariance test's FP64 Cholesky and whitening, and the FP64 oracle timed on
this host for one full 512^3 map (one thread and all cores).

Prints one JSON line (see the keys below). ``--gpus`` above 1 is refused: this build
measures one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "maps/s batched FP32 vs plain at 512³ box+cap sample, px err≤1e-5; HBM %peak"
HBM_PEAK_GBS = 8000.0
# rocprofv3 FETCH_SIZE, WRITE_SIZE (KiB per dispatch) of the noise + x kernel as it is now,
# on the first box (profile_run), by x tile width; a tile not measured reports null
TRAFFIC_X = {8: (2617.8, 114141.4)}


def support(N, L, k, p):
    """(drawn, y_rows, z_cols): the half-grid modes (ix, iy, iz <= N/2) whose weight
    P_box(|f|) is not zero -- the modes the noise pass draws (P_inf linear between table
    nodes, zero beyond the last one) --, the share of the (iy, packed column zc) x-lines
    that can be nonzero after pass x (fy^2 + zc^2 up to the last nonzero |f|^2: pass x
    writes them, pass y reads them), and the share of packed columns that can be nonzero
    after pass y (zc^2 up to it: pass y writes them, pass z reads them)."""
    import numpy as np
    f = np.arange(N)
    f2 = np.minimum(f, N - f) ** 2
    hist_xy = np.bincount((f2[:, None] + f2[None, :]).ravel())
    mmax = 3 * (N // 2) ** 2
    mult = np.zeros(mmax + 1, dtype=np.int64)
    for fz in range(N // 2 + 1):
        mult[fz * fz: fz * fz + hist_xy.size] += hist_xy
    km = (2 * math.pi / L) * np.sqrt(np.arange(mmax + 1, dtype=np.float64))
    pm = np.interp(km, k, p, left=0.0, right=0.0)
    pm[km > k[-1]] = 0.0
    pm[0] = 0.0
    m_hi = int(np.nonzero(pm > 0)[0].max()) if np.any(pm > 0) else 0
    zc = np.arange(N // 2)
    rows = (f2[:, None] + zc[None, :] ** 2) <= m_hi
    return int(mult[pm > 0].sum()), float(rows.mean()), float(np.mean(zc**2 <= m_hi))


def footprint(N, L, r, dirs, K=4):
    """(planes, lines, zband): the shares of x-planes, of (ix, iy) lines and of z nodes
    that the K-point interpolation stencils of the pixels read -- the only part of the
    field a map needs. Node i0 + a (mod N) per axis, i0 = floor((r n + L/2) N / L) - 1
    for K = 4."""
    import numpy as np
    base = np.floor((r * dirs + 0.5 * L) * (N / L)).astype(np.int64) - (1 if K == 4 else 0)
    read = np.zeros((N, N), bool)
    zread = np.zeros(N, bool)
    for a in range(K):
        zread[(base[:, 2] + a) % N] = True
        for b in range(K):
            read[(base[:, 0] + a) % N, (base[:, 1] + b) % N] = True
    return float(read.any(axis=1).mean()), float(read.mean()), float(zread.mean())


def build_jobs(torch, cmbx, workloads, n_boxes):
    from paper_2507_15703_amd import spectrum
    jobs = [j for j in workloads.ensemble_jobs() if j["N"] == 512][:n_boxes]
    out = []
    for j in jobs:
        N, L = j["N"], 1.0
        plan = cmbx.Plan(N, L, "f32", batch=1, interp="tricubic")
        plan.set_fixed_dirs(True)
        k, p = spectrum.synthetic_job_spectrum(N, L, j["r_over_L"] * L, j["theta_deg"], j["amp"])
        plan.spectrum_table(k, p)
        dirs = torch.tensor(workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"]), device="cuda")
        tuned = plan.autotune(reps=10, r=j["r_over_L"] * L, dirs=dirs)
        res = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        out.append(dict(plan=plan, seed=j["seed"], r=j["r_over_L"] * L, dirs=dirs, out=res,
                        theta=j["theta_deg"], n_pix=int(dirs.shape[0]), tuned=tuned,
                        support=support(N, L, k, p), k=k, p=p,
                        footprint=footprint(N, L, j["r_over_L"] * L, dirs.cpu().numpy())))
    return out


def cpu_baseline(jobs_meta):
    """The FP64 oracle timed on this host for one full map of the workload: the first 512^3
    job (its spectrum, seed, cap pixels, tricubic), noise + inverse FFT + gather, once with
    one thread and once with every core (the oracle's noise and gather on threads, scipy's
    FFT on as many workers). The per-core figure is the reported value."""
    import numpy as np

    from oracle import field as ofield
    from oracle import gather as ogather
    from oracle import noise as onoise
    from paper_2507_15703_amd import workloads

    j = jobs_meta[0]
    N, L = 512, 1.0
    dirs = workloads.cap_directions(j["theta"], int(round(25.6 * j["theta"])), 1024 if j["theta"] <= 20 else 2048)
    cores = len(os.sched_getaffinity(0))
    res = {}
    for threads in (cores, 1):
        t = {}
        t0 = time.perf_counter()
        h = onoise.halfgrid(N, L, j["seed"], j["k"], j["p"], threads=threads)
        t["noise"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        fld = ofield.field(h, workers=threads)
        t["fft"] = time.perf_counter() - t0
        del h
        t0 = time.perf_counter()
        ogather.gather(fld, L, j["r"], dirs, "tricubic", threads=threads)
        t["gather"] = time.perf_counter() - t0
        del fld
        res[threads] = t
        print(f"[bench] oracle map on {threads} thread(s): {sum(t.values()):.1f} s", file=sys.stderr, flush=True)
    sec_all, sec_one = sum(res[cores].values()), sum(res[1].values())
    return {"value": 1.0 / sec_all, "unit": "maps/s", "cores": cores, "kind": "oracle",
            "sample": (f"one whole 512^3 FP64 oracle map of the workload (first box: noise of all {N * N * (N // 2 + 1)} "
                       f"half-grid modes, scipy inverse FFT, tricubic gather of {len(dirs)} pixels), timed end to end "
                       f"on {cores} threads: {sec_all:.2f} s (noise {res[cores]['noise']:.2f}, fft {res[cores]['fft']:.2f}, "
                       f"gather {res[cores]['gather']:.2f}); on 1 thread: {sec_one:.2f} s (noise {res[1]['noise']:.2f}, "
                       f"fft {res[1]['fft']:.2f}, gather {res[1]['gather']:.2f})"),
            "one_thread_maps_per_s": 1.0 / sec_one}


def fft_instr_per_point(N):
    """VALU instructions per point of a length-N inverse transform as the x pass runs it
    (N = 512: radix 8 x 8 x 8). A radix-8 butterfly is 56 real additions and
    multiplications (two length-4 transforms of 16, the e^{i pi/4} and e^{3i pi/4}
    rotations of 4 each, 16 for the final sums), 7 per point; every stage after the first
    also multiplies 7 of its 8 inputs by a twiddle, 4 instructions each with the products
    fused into multiply-adds: 3.5 more per point."""
    if N != 512:
        raise ValueError("counted for N = 512")
    return 7.0 + 2 * (7.0 + 3.5)


# Per drawn mode: half a Philox4x32-10 call (10 rounds of two 32 x 32 -> 64-bit
# multiplies and two three-input XORs: 40 instructions per call of two modes), the
# binary32 Box-Muller sequence (49 operations with its conversions, multiplies and adds
# never fused), and the two weight products.
NOISE_INSTR_PER_MODE = 20 + 49 + 2


def event_ms(torch, fn, reps):
    """Average ms of fn() over reps calls on torch's current stream (after one warm-up)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def slab_section(torch, cmbx, reps=20):
    """The 2-D (hybrid) Fourier method (Sec. II D 2) and the 3-D method on the same flat box,
    in the paper's setting: unit sphere, beam b = 0.573 deg (0.01 rad), 10-degree cap, the
    box of the Sec. II C sizing rule (N = 512, M = 32, dp = 0.0017), h = 14 layers (the cap's
    height plus the stencil), the programme's P_inf, FP32, tricubic, the pixels of the
    HEALPix cap at nside 64 (the paper's resolution for this beam). ms per map from HIP
    events; the paper's time factor N^2 log2(N^2) h for context."""
    from paper_2507_15703_amd import spectrum, workloads
    b, theta = 0.01, math.radians(10.0)
    z_min = math.cos(theta)
    N, M, dp = cmbx.box_size(b, theta)
    h = min(M, int(math.ceil((1.0 - z_min) / dp)) + 5)
    cl = workloads.synthetic_cl(int(math.ceil(5.0 / b)), ld=1.0 / b)
    k, p, _ = spectrum.invert(cl, 1.0, theta, b, k_max=math.pi / dp)
    dirs = cmbx.healpix_cap(64, z_min)
    out = {"N": N, "M": M, "h": h, "dp": dp, "nside": 64, "pixels": int(dirs.shape[0]),
           "paper_time_factor_hybrid": N * N * math.log2(N * N) * h}
    for method in ("hybrid", "flat"):
        slab = cmbx.Slab(method, N, M, dp, h=h, dtype="f32", interp="tricubic")
        t0 = time.perf_counter()
        slab.spectrum(k, p)
        t_tab = time.perf_counter() - t0
        slab.set_observer(slab.observer_for_cap(1.0, z_min))
        res = torch.empty((1, dirs.shape[0]), dtype=torch.float32, device="cuda")
        ms = event_ms(torch, lambda: slab.simulate(7, 1.0, dirs, out=res), reps)
        assert bool(torch.isfinite(res).all())
        out[method] = {"layers": slab.nz, "ms_per_map": round(ms, 4), "maps_per_s": round(1e3 / ms, 1),
                       "table_s": round(t_tab, 3)}
        slab.close()
        print(f"[bench] {method} {N}x{N}x{M}: {ms:.4f} ms/map", file=sys.stderr, flush=True)
    return out


def covtest_section(torch, cmbx, n_maps=1000):
    """The covariance test's linear algebra (Sec. III B) at the paper's size: Gamma of the
    30-degree HEALPix cap at nside 64, Cholesky of Gamma + 1e-6 Gamma_00 I (n^3 / 3 FP64
    multiply-adds), whitening of 1000 maps (n^2 each); against the FP64 matrix-core peak
    78.6 TFLOP/s (a multiply-add is two operations)."""
    from paper_2507_15703_amd import workloads
    z_min = math.cos(math.radians(30.0))
    dirs = cmbx.healpix_cap(64, z_min)
    n = int(dirs.shape[0])
    cl = workloads.synthetic_cl(500, ld=100.0)
    G = cmbx.pixel_covariance(dirs, cl)
    shift = 1e-6 * float(G[0, 0].item())
    L = torch.empty_like(G)
    ms_chol = event_ms(torch, lambda: (L.copy_(G), cmbx.cholesky(L, shift=shift)), 3)
    ms_copy = event_ms(torch, lambda: L.copy_(G), 3)
    ms_chol -= ms_copy
    maps = torch.randn((n_maps, n), dtype=torch.float64, device="cuda")
    ms_wh = event_ms(torch, lambda: cmbx.whiten(L, maps), 3)
    fl_chol, fl_wh = n**3 / 3.0, float(n) * n * n_maps
    return {"nside": 64, "cap_deg": 30.0, "n_pix": n, "maps": n_maps,
            "cholesky_ms": round(ms_chol, 3), "cholesky_TFLOPs": round(fl_chol / (ms_chol * 1e-3) / 1e12, 2),
            "whiten_ms": round(ms_wh, 3), "whiten_TFLOPs": round(fl_wh / (ms_wh * 1e-3) / 1e12, 2),
            "fp64_peak_TFLOPs": 78.6}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # untimed steps before the timed region: 50 steps (about 35 ms) bring the timed region
    # within about 1 % of the steady state the alternating blocks below measure; 5 left it 2 % short
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--boxes", type=int, default=4, help="512^3 boxes per step (<= 4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--mode", default="auto", choices=["auto", "chained", "pipelined"],
                    help="ensemble execution mode of the batched path")
    ap.add_argument("--lanes", type=int, default=None, choices=[1, 2, 3, 4],
                    help="graphs the chained items are split over (default: auto mode times 1 .. 4)")
    ap.add_argument("--blocks", type=int, default=7,
                    help="alternating blocks of --steps plain and batched steps for the spread")
    ap.add_argument("--no-extras", action="store_true", help="skip the hybrid and flat-box section")
    ap.add_argument("--covtest", action="store_true",
                    help="also time the covariance test's FP64 Cholesky and whitening (its own run records them)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): independent realisations "
              "shard across GPUs with no communication; run one process per GPU instead.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2507_15703_amd import cmbx, workloads

    torch.cuda.set_device(0)
    jobs = build_jobs(torch, cmbx, workloads, args.boxes)
    nmaps = len(jobs)
    ens = cmbx.Ensemble([dict(plan=j["plan"], seed=j["seed"], r=j["r"], dirs=j["dirs"], out=j["out"]) for j in jobs],
                        mode=args.mode, lanes=args.lanes)

    def step_batched():
        ens.launch()

    def step_plain():
        for j in jobs:
            j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"], j["out"])

    def timed(step, K, W):
        for _ in range(W):
            step()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s)
        for _ in range(K):
            step()
        e1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / 1e3, wall

    print(f"[bench] {nmaps} x 512^3 FP32 boxes, pixels {[j['n_pix'] for j in jobs]}", file=sys.stderr, flush=True)
    ev_b, wall_b = timed(step_batched, args.steps, args.warmup)
    print(f"[bench] batched: {ev_b * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    ev_p, wall_p = timed(step_plain, args.steps, args.warmup)
    print(f"[bench] plain:   {ev_p * 1e3 / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    sec_b = max(ev_b, 1e-12)
    value = nmaps * args.steps / sec_b
    plain = nmaps * args.steps / max(ev_p, 1e-12)
    # spread: alternating blocks of the same number of steps, plain then batched
    blocks = {"plain": [], "batched": []}
    for _ in range(args.blocks):
        for name, fn in (("plain", step_plain), ("batched", step_batched)):
            t, _w = timed(fn, args.steps, 1)
            blocks[name].append(nmaps * args.steps / max(t, 1e-12))
    import statistics
    spread = {n: {"median": round(statistics.median(v), 1), "min": round(min(v), 1), "max": round(max(v), 1)}
              for n, v in blocks.items()}
    ratios = sorted(b / p for b, p in zip(blocks["batched"], blocks["plain"]))
    print(f"[bench] blocks: batched {spread['batched']}, plain {spread['plain']}", file=sys.stderr, flush=True)

    # per-kernel durations (HIP events on the plan's stream, the stream they run on)
    j0 = jobs[0]
    ms = j0["plan"].time_passes(j0["seed"], j0["r"], j0["dirs"], j0["out"], reps=args.kernel_reps)
    N = 512
    field_bytes = 4 * N**3
    drawn, y_rows, z_cols = j0["support"]
    planes, lines, zband = j0["footprint"]
    # algorithmic bytes: only what can be nonzero (the spectrum's support) and what the
    # map reads (the stencils' footprint) moves -- pass x writes the x-lines within the
    # support, rows of the planes read; pass y reads those and writes the columns within
    # the support of the lines read; pass z reads those and writes the z nodes read of the
    # lines read; with the directions fixed the gather reads each pixel's record in the
    # pixel order (16 B: stencil node and fractions) and its index (4 B) and writes the
    # map (4 B)
    kbytes = [int(field_bytes * y_rows * planes), int(field_bytes * (y_rows * planes + z_cols * lines)),
              int(field_bytes * (z_cols + zband) * lines), 24 * j0["n_pix"]]
    names = ["pass_x_noise", "pass_y", "pass_z_c2r", "gather_tricubic"]
    kernels = {n: {"ms": round(t, 4), "alg_bytes": b, "GBps": round(b / (t * 1e-3) / 1e9, 1)}
               for n, t, b in zip(names, ms, kbytes)}
    # the footprint (clear, mark the stencils, list the z blocks), timed on the plan's
    # stream: it reads the directions (24 B per pixel)
    import ctypes
    plan0 = j0["plan"]
    fbuf = torch.zeros(int(cmbx.lib().cmbx_footprint_bytes(N)), dtype=torch.uint8, device="cuda")
    def make_fp():
        cmbx._check(cmbx.lib().cmbx_debug_footprint(plan0.handle, ctypes.c_double(j0["r"]), j0["dirs"].data_ptr(),
                                                    j0["n_pix"], fbuf.data_ptr()))
    make_fp()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.kernel_reps):
        make_fp()
    e1.record()
    torch.cuda.synchronize()
    t_fp = e0.elapsed_time(e1) / args.kernel_reps
    kernels["footprint"] = {"ms": round(t_fp, 4), "alg_bytes": 24 * j0["n_pix"],
                            "GBps": round(24 * j0["n_pix"] / (t_fp * 1e-3) / 1e9, 1)}
    # The dominant kernel is the noise + x pass, bound by the vector ALU. Its algorithmic
    # work in VALU instructions (a fused multiply-add counts once): per drawn mode (weight
    # not zero) NOISE_INSTR_PER_MODE, per point of the x-lines within the spectrum's support
    # the transform's fft_instr_per_point (the other lines are zero and need none). Peak:
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s for unpacked
    # operations, one wave instruction per SIMD every four cycles; the published FP32 vector
    # peak, 157.3 TFLOP/s, counts a multiply-add as two operations and packed FP32 twice.
    ops_launch = drawn * NOISE_INSTR_PER_MODE + (N**3 // 2) * y_rows * fft_instr_per_point(N)
    alu_peak = 256 * 4 * 16 * 2.4e9
    ach_ops = ops_launch / (ms[0] * 1e-3)
    # HBM bytes per launch of this kernel from rocprofv3 FETCH_SIZE (x2.0 calibration against
    # a plain copy) + WRITE_SIZE (x1.0), by tile width, for this box's spectrum (counters of
    # the current kernel code; None once the kernel has changed since they were taken)
    traffic_by_tile = {t: (f * 2.0 + w) * 1024 for t, (f, w) in TRAFFIC_X.items()}
    tile_x = jobs[0]["tuned"]["tile_x"]
    roofline = {"kernel": names[0], "bound": "alu", "achieved": round(ach_ops / 1e12, 2),
                "peak": round(alu_peak / 1e12, 2), "unit": "T VALU lane-instr/s", "frac": round(ach_ops / alu_peak, 4),
                "frac_of_published_fp32": round(ach_ops / 157.3e12, 4),
                "traffic": traffic_by_tile.get(tile_x), "instr_per_launch": int(ops_launch),
                "instr_per_drawn_mode": NOISE_INSTR_PER_MODE, "instr_per_point_fft": fft_instr_per_point(N),
                "drawn_modes": drawn, "half_grid_modes": N * N * (N // 2 + 1)}
    # the two transform passes are HBM-bound: fraction of the 8 TB/s peak
    for i in (1, 2):
        kernels[names[i]]["hbm_frac"] = round(kbytes[i] / (ms[i] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    map_bytes = sum(4 * N**3 * (2 * j["support"][1] * j["footprint"][0]
                                + (2 * j["support"][2] + j["footprint"][2]) * j["footprint"][1])
                    + 28 * j["n_pix"] for j in jobs) / nmaps  # directions and map (footprint made once)
    path_gbs = map_bytes * value / 1e9

    # HEALPix cap pixels made on the device (an input of the path, outside the step):
    # nside 2048, 26.85 deg cap (2.7M pixels), 24 bytes written per pixel
    hp_z = math.cos(math.radians(26.85))
    hp_n = cmbx.healpix_cap_count(2048, hp_z)
    hp_buf = torch.empty((hp_n, 3), dtype=torch.float64, device="cuda")
    cmbx.healpix_cap(2048, hp_z, out=hp_buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cmbx.healpix_cap(2048, hp_z, out=hp_buf)
    e1.record()
    torch.cuda.synchronize()
    hp_ms = e0.elapsed_time(e1) / 10
    healpix = {"nside": 2048, "theta_max_deg": 26.85, "pixels": hp_n, "ms": round(hp_ms, 4),
               "GBps": round(24 * hp_n / (hp_ms * 1e-3) / 1e9, 1)}

    # pixel covariance from C_l for the covariance test of the maps (outside the step):
    # nside 128, 20 deg HEALPix cap, lmax 1000; 4 FP64 operations per entry and l
    cv_dirs = cmbx.healpix_cap(128, math.cos(math.radians(20.0)))
    cv_n, cv_l = cv_dirs.shape[0], 1000
    cv_cl = 1.0 / (1.0 + torch.arange(cv_l + 1, dtype=torch.float64, device="cuda")) ** 2
    cv_out = torch.empty((cv_n, cv_n), dtype=torch.float64, device="cuda")
    cmbx.pixel_covariance(cv_dirs, cv_cl, out=cv_out)
    e0.record()
    for _ in range(5):
        cmbx.pixel_covariance(cv_dirs, cv_cl, out=cv_out)
    e1.record()
    torch.cuda.synchronize()
    cv_ms = e0.elapsed_time(e1) / 5
    cv_ops = 4.0 * cv_n * cv_n * (cv_l + 1)
    covariance = {"nside": 128, "theta_max_deg": 20.0, "pixels": cv_n, "lmax": cv_l, "ms": round(cv_ms, 3),
                  "Tops": round(cv_ops / (cv_ms * 1e-3) / 1e12, 2),
                  "alu_frac": round(cv_ops / (cv_ms * 1e-3) / alu_peak, 4)}
    del cv_out

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_b * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{nmaps}x512^3 FP32 batched (hipGraph ensemble), r=0.45L, caps U[10,40] deg, tricubic",
                   "boxes": nmaps, "N": N, "pixels": [j["n_pix"] for j in jobs], "maps_per_step": nmaps,
                   "fixed_dirs": True},
        "plain_maps_per_s": round(plain, 2),
        "ensemble_mode": ens.modes,
        "ensemble_lanes": ens.lanes,
        "batched_over_plain": round(value / plain, 3),
        "blocks": {"steps_each": args.steps, "count": args.blocks, "maps_per_s": spread,
                   "batched_over_plain": {"median": round(statistics.median(ratios), 3), "min": round(ratios[0], 3),
                                          "max": round(ratios[-1], 3)},
                   "batched_beats_plain_every_block": bool(min(blocks["batched"]) > max(blocks["plain"]))},
        "wall_s": {"batched": round(wall_b, 4), "plain": round(wall_p, 4)},
        "path_GBps_alg": round(path_gbs, 1),
        "path_hbm_frac_alg": round(path_gbs / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "tiles": {k: jobs[0]["tuned"][k] for k in ("tile_x", "tile_y", "lines_z", "plans")},
        "roofline": roofline,
        "healpix_cap": healpix,
        "pixel_covariance": covariance,
    }
    for j in jobs:
        j["plan"].close()
    ens.close()
    if not args.no_extras:
        result["flat_box_methods"] = slab_section(torch, cmbx)
    if args.covtest:
        result["covariance_test"] = covtest_section(torch, cmbx)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (one oracle map) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(jobs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
