"""A short, fixed launch sequence for rocprofv3 (kernel trace and counter passes).

Runs, on one FP32 plan of the benchmark's first 512^3 box (tricubic, r = 0.45 L, its cap
of 26.9 deg and 687 x 2048 pixels, its spectrum: the programme's solution for the synthetic
C_l on that cap, ``spectrum.synthetic_job_spectrum``; the power-law table with
``--spectrum powerlaw``; autotuned tile shapes unless given; directions fixed, as the
benchmark runs them), with its seed: one
warm-up realisation, then ``--reps`` launches of each kernel of the hot path through
cmbx_time_passes, and a device-to-device copy of exactly 512 MiB (torch) whose counter
readings calibrate the HBM byte counters. With ``--slab``: instead, the benchmark's
flat-box section (the 2-D method and the 3-D method on the flat N = 512, M = 32 box of a
10-degree cap, h = 14 layers, nside-64 pixels), ``--reps`` maps of each. With
``--ensemble``: the benchmark's four 512^3 boxes as its batched path runs them (chained on
two lanes, directions fixed), ``--reps`` launches after two warm-up launches, for the
time kernels of the two lanes share the chip (``trace_overlap``). Usage:

    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2507_15703_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_2507_15703_amd.profile_run --reps 1
    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2507_15703_amd.profile_run --slab
    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2507_15703_amd.profile_run --ensemble
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--tile-xy", type=int, default=0)
    ap.add_argument("--lines-z", type=int, default=0)
    ap.add_argument("--plans", default=None, help="FFT stage plans of x, y, z as 'a,b,c' (with given tiles)")
    ap.add_argument("--tile-y", type=int, default=None)
    ap.add_argument("--spectrum", default="lp", choices=["lp", "powerlaw"])
    ap.add_argument("--slab", action="store_true", help="the flat-box methods instead")
    ap.add_argument("--ensemble", action="store_true", help="the benchmark's batched path instead")
    args = ap.parse_args()

    import torch

    from paper_2507_15703_amd import cmbx, spectrum, workloads
    if args.slab:
        import bench
        print(json.dumps(bench.slab_section(torch, cmbx, reps=args.reps)), flush=True)
        return
    if args.ensemble:
        import bench
        jobs = bench.build_jobs(torch, cmbx, workloads, 4)
        ens = cmbx.Ensemble([dict(plan=j["plan"], seed=j["seed"], r=j["r"], dirs=j["dirs"], out=j["out"]) for j in jobs],
                            mode="chained", lanes=2)
        for _ in range(2):
            ens.launch()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.reps):
            ens.launch()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.reps
        print(json.dumps({"boxes": len(jobs), "lanes": ens.lanes, "ms_per_launch": round(ms, 4),
                          "maps_per_s": round(len(jobs) / ms * 1e3, 1)}), flush=True)
        ens.close()
        return

    N = args.N
    job = [j for j in workloads.ensemble_jobs() if j["N"] == 512][0]
    plan = cmbx.Plan(N, 1.0, args.dtype, batch=1, interp="tricubic")
    plan.set_fixed_dirs(True)  # as bench.py: footprint made once, the gather in pixel order
    if args.spectrum == "lp":
        k, p = spectrum.synthetic_job_spectrum(N, 1.0, job["r_over_L"], job["theta_deg"], job["amp"])
    else:
        k, p = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=N / 4)
    plan.spectrum_table(k, p)
    dirs = torch.tensor(workloads.cap_directions(job["theta_deg"], job["n_ring"], job["n_phi"]), device="cuda")
    if args.tile_xy or args.lines_z or args.plans:
        plans = tuple(int(v) for v in args.plans.split(",")) if args.plans else None
        plan.set_tiles(args.tile_xy, args.lines_z, tile_y=args.tile_y, plans=plans)
    else:
        plan.autotune(reps=10, r=job["r_over_L"], dirs=dirs)  # as bench.py tunes
    out = torch.empty((1, dirs.shape[0]), dtype=plan.torch_dtype, device="cuda")
    seed, r = job["seed"], job["r_over_L"]
    plan.simulate_patch(seed, r, dirs, out)
    torch.cuda.synchronize()
    ms = plan.time_passes(seed, r, dirs, out, reps=args.reps)
    src = torch.ones(512 * 2**20 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"N": N, "dtype": args.dtype, "reps": args.reps, "pixels": int(dirs.shape[0]),
                      "shapes": plan.shapes(),
                      "ms": {"pass_x": ms[0], "pass_y": ms[1], "pass_z": ms[2], "gather": ms[3]},
                      "copy_bytes": 2 * 512 * 2**20}), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
