"""Train the C_l -> P_inf surrogate on pairs from the plain inversion and report on it.

    python -m paper_2507_15703_amd.train_surrogate --pairs 50000 --data pairs.npz \
        --out surrogate_state.npz [--export weights.npz] [--steps 20000] [--resume state.npz]

Pairs (features, targets) are generated with the host inversion on all host cores and
cached in --data (reused when present). Training runs on the GPU through the library's
MLP kernels; --out keeps the full training state (FP32 masters, Adam moments, step; with
a CRC) and --export the BF16 weights inference loads. Held-out spectra (seeds 5000 ..)
at --eval-N, --eval-r measure the share that passes every check (bands after the projection
within --tol; in-cap correlations no more than --res-tol of xi(0) below the target and
--exc-tol above it), the correlation deficits of the network's answers next to those of
the spectrum-independent mean target, and spectra/s of
network + projection + checks against the linear programme. Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--data", default="surrogate_pairs.npz")
    ap.add_argument("--out", default="surrogate_state.npz")
    ap.add_argument("--export", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--eval-N", type=int, default=256)
    ap.add_argument("--eval-r", type=float, default=0.45)
    ap.add_argument("--tol", type=float, default=0.01)
    ap.add_argument("--res-tol", type=float, default=0.002)
    ap.add_argument("--exc-tol", type=float, default=0.02)
    args = ap.parse_args()

    from paper_2507_15703_amd import surrogate

    t0 = time.time()
    if os.path.exists(args.data):
        d = np.load(args.data)
        X, Y = d["X"], d["Y"]
        if X.shape[0] < args.pairs:
            Xa, Ya = surrogate.generate_pairs(args.pairs - X.shape[0], seed=1_000_000 + X.shape[0])
            X, Y = np.concatenate([X, Xa]), np.concatenate([Y, Ya])
            np.savez(args.data, X=X, Y=Y)
        X, Y = X[: args.pairs], Y[: args.pairs]
    else:
        X, Y = surrogate.generate_pairs(args.pairs, seed=1_000_000)
        np.savez(args.data, X=X, Y=Y)
    t_data = time.time() - t0
    print(f"[train] {X.shape[0]} pairs ready in {t_data:.1f} s", file=sys.stderr, flush=True)

    net = surrogate.MLP(seed=0)
    if args.resume:
        net.load_state(surrogate.read_checkpoint(args.resume))
    t0 = time.time()
    losses = net.train(X, Y, steps=args.steps, batch=args.batch, lr=args.lr, log_every=max(1, args.steps // 10),
                       seed=net.step)
    t_train = time.time() - t0
    for it, l in losses:
        print(f"[train] step {it} loss {l:.4g}", file=sys.stderr, flush=True)
    # the mean training target travels with the weights: the network-free baseline the
    # surrogate study measures the network against
    y_prior = Y.mean(axis=0).astype(np.float32)
    surrogate.save_checkpoint(args.out, net.state() | {"y_prior": y_prior})
    if args.export:
        surrogate.save_checkpoint(args.export, net.inference_state() | {"y_prior": y_prior})

    # held-out spectra at the evaluation geometry
    items = []
    for s in range(5000, 5000 + args.eval):
        prm = surrogate.sample_params(np.random.default_rng(s))
        prm["N"], prm["r"] = args.eval_N, args.eval_r
        prm["ld"] = float(np.random.default_rng(s + 77).uniform(0.4, 0.8)) * surrogate.lmax_of(prm["N"], prm["r"])
        items.append((surrogate.cl_of(prm), prm["N"], prm["r"]))
    sur = surrogate.Surrogate(net, tol=float("inf"), res_tol=float("inf"), exc_tol=float("inf"))  # keep every answer
    sur.spectra(items[:1])
    t0 = time.perf_counter()
    got = sur.spectra(items)
    t_net = time.perf_counter() - t0
    dev = np.array([g[3][0] for g in got])
    res = np.array([g[3][1] for g in got])
    exc = np.array([g[3][2] for g in got])
    # the same projection and checks started from the mean training target instead of the network
    res_mean = np.array([sur.answer(y_prior, *it)[2][1] for it in items])
    t_lp = 0.0
    n_lp = min(8, len(items))
    for cl, N, r in items[:n_lp]:
        t1 = time.perf_counter()
        surrogate.spectrum.invert(cl, r * surrogate.L_BOX, surrogate.THETA_MAX, 1.0 / (0.6 * (cl.size - 1)), N=N)
        t_lp += time.perf_counter() - t1
    out = {"pairs": int(X.shape[0]), "steps": args.steps, "final_loss": losses[-1][1], "train_s": round(t_train, 1),
           "data_s": round(t_data, 1), "eval": args.eval, "eval_N": args.eval_N, "eval_r": args.eval_r,
           "band_dev_max": float(dev.max()), "corr_deficit_median": float(np.median(res)),
           "corr_deficit_p90": float(np.percentile(res, 90)), "corr_deficit_median_mean_prior": float(np.median(res_mean)),
           "corr_excess_max": float(exc.max()),
           "accepted_frac": float(np.mean((dev <= args.tol) & (res <= args.res_tol) & (exc <= args.exc_tol))),
           "accepted_frac_mean_prior": float(np.mean(res_mean <= args.res_tol)), "tol": args.tol,
           "res_tol": args.res_tol, "exc_tol": args.exc_tol,
           "net_spectra_per_s": round(len(items) / t_net, 1), "lp_spectra_per_s": round(n_lp / t_lp, 2),
           "state": args.out, "weights": args.export}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
