"""Throughput of the mixed-size ensemble, batched against unbatched, on one GPU.

    python -m paper_2507_15703_amd.ensemble_run [--steps 10] [--warmup 2] [--dtype f32] [--fixed-dirs]

The ensemble workload: 16 x 128^3 + 8 x 256^3 + 4 x 384^3 + 4 x 512^3 boxes, each with
its own seed, r = 0.45 L, a cap of half-angle drawn in [10, 40] deg and a spectrum
amplitude drawn in [0.8, 1.2] (``workloads.ensemble_jobs``), tricubic; each box's P(k) is
the programme's solution for the synthetic C_l family on its cap (host inversion,
``spectrum.synthetic_job_spectrum``; ``--spectrum powerlaw`` takes the power-law table).
One step maps every box once. The batched path is one ``cmbx.Ensemble`` (auto mode: per size group the
faster of chained and pipelined, one or two lanes); the unbatched path calls
``simulate_patch`` job after job on one stream. Tile shapes are autotuned per box on its
own pixels.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def build(torch, cmbx, workloads, dtype, kind="lp", fixed_dirs=False):
    from paper_2507_15703_amd import spectrum
    jobs = []
    for j in workloads.ensemble_jobs():
        N, L = j["N"], 1.0
        plan = cmbx.Plan(N, L, dtype, batch=1, interp="tricubic")
        if fixed_dirs:
            plan.set_fixed_dirs(True)
        if kind == "lp":
            k, p = spectrum.synthetic_job_spectrum(N, L, j["r_over_L"] * L, j["theta_deg"], j["amp"])
        else:
            k, p = workloads.powerlaw_cutoff_table(N, L, kc_modes=N / 4)
            p = p * j["amp"]
        plan.spectrum_table(k, p)
        dirs = torch.tensor(workloads.cap_directions(j["theta_deg"], j["n_ring"], j["n_phi"]), device="cuda")
        plan.autotune(reps=3, r=j["r_over_L"] * L, dirs=dirs)
        out = torch.empty((1, dirs.shape[0]), dtype=plan.torch_dtype, device="cuda")
        jobs.append(dict(plan=plan, seed=j["seed"], r=j["r_over_L"] * L, dirs=dirs, out=out, N=N))
    return jobs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--spectrum", default="lp", choices=["lp", "powerlaw"])
    ap.add_argument("--fixed-dirs", action="store_true",
                    help="every plan keeps its directions (one footprint per plan, as in bench.py)")
    args = ap.parse_args()

    import torch

    from paper_2507_15703_amd import cmbx, workloads

    jobs = build(torch, cmbx, workloads, args.dtype, args.spectrum, args.fixed_dirs)
    ens = cmbx.Ensemble([{k: j[k] for k in ("plan", "seed", "r", "dirs", "out")} for j in jobs], mode="auto")

    def batched():
        ens.launch()

    def plain():
        for j in jobs:
            j["plan"].simulate_patch(j["seed"], j["r"], j["dirs"], j["out"])

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.steps):
            step()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    t_b = timed(batched)
    t_p = timed(plain)
    n = len(jobs) * args.steps
    sizes = sorted({j["N"] for j in jobs})
    print(json.dumps({"workload": "16x128^3 + 8x256^3 + 4x384^3 + 4x512^3, caps U[10,40] deg, tricubic",
                      "spectrum": args.spectrum, "dtype": args.dtype, "fixed_dirs": args.fixed_dirs, "maps_per_step": len(jobs), "steps": args.steps,
                      "batched_maps_per_s": round(n / t_b, 1), "plain_maps_per_s": round(n / t_p, 1),
                      "batched_over_plain": round(t_p / t_b, 3), "ms_per_step_batched": round(t_b / args.steps * 1e3, 3),
                      "groups": dict(zip(sizes, ens.modes)), "lanes": ens.lanes,
                      "pixels": sum(int(j["dirs"].shape[0]) for j in jobs)}), flush=True)
    ens.close()
    for j in jobs:
        j["plan"].close()


if __name__ == "__main__":
    main()
