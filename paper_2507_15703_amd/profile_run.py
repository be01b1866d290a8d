"""A short, fixed launch sequence for rocprofv3 (kernel trace and counter passes).

Runs, on one 512^3 FP32 plan (tricubic, r = 0.45 L, 30 deg cap of 768 x 2048 pixels,
spectrum from the programme for the synthetic C_l on that cap as in the benchmark, or the
power-law table with ``--spectrum powerlaw``; autotuned tile shapes unless given): one
warm-up realisation, then ``--reps`` launches of each kernel of the hot path through
cmbx_time_passes, and a device-to-device copy of exactly 512 MiB (torch) whose counter
readings calibrate the HBM byte counters. Usage:

    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2507_15703_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_2507_15703_amd.profile_run --reps 1
"""
import argparse
import json
import math
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
    ap.add_argument("--spectrum", default="lp", choices=["lp", "powerlaw"])
    args = ap.parse_args()

    import torch

    from paper_2507_15703_amd import cmbx, spectrum, workloads

    N = args.N
    plan = cmbx.Plan(N, 1.0, args.dtype, batch=1, interp="tricubic")
    if args.spectrum == "lp":
        lmax = workloads.lmax_for(N, 1.0, 0.45)
        k, p, _ = spectrum.invert(workloads.synthetic_cl(lmax), 0.45, math.radians(30.0), 1.0 / (0.6 * lmax), N=N)
    else:
        k, p = workloads.powerlaw_cutoff_table(N, 1.0, kc_modes=N / 4)
    plan.spectrum_table(k, p)
    if args.tile_xy or args.lines_z:
        plan.set_tiles(args.tile_xy, args.lines_z)
    else:
        plan.autotune(reps=3)  # the tile shapes bench.py uses
    dirs = torch.tensor(workloads.cap_directions(30.0, 768, 2048), device="cuda")
    out = torch.empty((1, dirs.shape[0]), dtype=plan.torch_dtype, device="cuda")
    plan.simulate_patch(1, 0.45, dirs, out)
    torch.cuda.synchronize()
    ms = plan.time_passes(1, 0.45, dirs, out, reps=args.reps)
    src = torch.ones(512 * 2**20 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"N": N, "dtype": args.dtype, "reps": args.reps, "pixels": int(dirs.shape[0]),
                      "ms": {"pass_x": ms[0], "pass_y": ms[1], "pass_z": ms[2], "gather": ms[3]},
                      "copy_bytes": 2 * 512 * 2**20}), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
