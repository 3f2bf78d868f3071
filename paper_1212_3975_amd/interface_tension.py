"""Order-disorder interface tension of the 8-state Potts model (Sec. 5, Eq. 9).

Orchestration only (every step runs in libmuca.so).  For each lattice size:
  1. Seed the log-weights with the learned network, if parameters are given,
     or (--chain-seed) with the previous size's converged weights rescaled
     per site (ln W / N as a function of E / N carries over between sizes), or
     (--weights) with an earlier run's weights for the same size.
  2. Iterate the recursion, with the correction function, until the merged
     histogram is flat; then refine it with a few more iterations.
  3. Re-thermalise, then run production sweeps.
  4. Find the equal-height inverse temperature of the reweighted energy
     histogram, and sigma_od(L) = ln(P_max/P_min)/(2L) there.
Finally, fit sigma_od(L) = sigma_inf + a/L over the larger sizes.

  python -m paper_1212_3975_amd.interface_tension --out DIR [--params mlp_params.npy]
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

import paper_1212_3975_amd as pm  # noqa: E402
from paper_1212_3975_amd.learned_init import iterate_to_flat  # noqa: E402
from workloads import POTTS, Problem  # noqa: E402

BETA0 = math.log(1.0 + math.sqrt(8.0))   # Sec. 3: transition point of the 8-state Potts model


def fit_inverse_l(Ls, sigmas):
    """Least-squares sigma(L) = sigma_inf + a / L."""
    A = np.stack([np.ones(len(Ls)), 1.0 / np.asarray(Ls, np.float64)], axis=1)
    (s_inf, a), *_ = np.linalg.lstsq(A, np.asarray(sigmas, np.float64), rcond=None)
    return float(s_inf), float(a)


def rescaled_weights(lnW_prev, L_prev, L):
    """Per-site carry-over of converged log-weights: lnW_L(E) = N_L * w(E / N_L)
    with w(e) = lnW_prev(e N_prev) / N_prev, interpolated linearly in e."""
    Np, N = L_prev * L_prev, L * L
    e_prev = (-2.0 * Np + np.arange(2 * Np + 1)) / Np
    e_new = (-2.0 * N + np.arange(2 * N + 1)) / N
    return N * np.interp(e_new, e_prev, np.asarray(lnW_prev, np.float64) / Np)


def run_size(L, chains, seed, sweeps, cap, refine, n_therm, n_prod, mlp, max_seconds, seed_lnw=None, flat_rule=0,
             iterate=True, blocks=0):
    prob = Problem(POTTS, L, chains, seed, q=8)
    rec = {"L": L, "chains": chains, "seed": seed, "sweeps_per_iter": sweeps,
           "weights_seed": "given" if seed_lnw is not None else ("learned" if mlp is not None else "zero")}
    t0 = time.time()
    rec["flat_rule"] = "paper: [<H>/2, 2<H>]" if flat_rule == 1 else "min/max >= 0.5"
    with pm.Muca([prob], correction=1, flat_rule=flat_rule) as ctx:
        if seed_lnw is not None:
            ctx.set_log_weights(0, seed_lnw)
        elif mlp is not None:
            mlp.set_log_weights(ctx, 0)
        if iterate:
            n_flat, _ = iterate_to_flat(ctx, sweeps, cap, f"potts8 L={L}", log_every=10, max_seconds=max_seconds)
            rec["iterations_to_flat"] = n_flat
            if n_flat is None:
                rec["seconds"] = round(time.time() - t0, 1)
                return rec, None, None
            for _ in range(refine):
                ctx.iterate(sweeps)
        else:
            rec["iterations_to_flat"] = 0   # production on the given weights as they are
        lnW = ctx.lnW(0)
        ctx.sweep(n_therm, pm.REC_NONE)
        done = 0
        while done < n_prod:
            n = min(2000, n_prod - done)
            ctx.sweep(n, pm.REC_PROD)
            done += n
            ctx.stream.synchronize()
            print(f"  potts8 L={L} production {done}/{n_prod} t={time.time() - t0:.1f}s", flush=True)
        rec["production_sweeps"] = n_prod
        res = None
        for half in (0.02, 0.05, 0.1, 0.2):
            try:
                res = ctx.interface_tension(0, BETA0 - half, BETA0 + half)
                rec["bracket_half_width"] = half
                break
            except pm.MucaError as e:
                rec["last_error"] = str(e)
        rec["seconds"] = round(time.time() - t0, 1)
        if res is None:
            return rec, None, lnW
        rec.update(beta_eqh=res["beta"], sigma_od=res["sigma"], k_peaks=list(res["k_peaks"]),
                   ln_ratio=res["sigma"] * 2 * L)
        if blocks:
            # the same analysis on disjoint blocks of chains (each block's merged
            # production counts, the run's weights): how much of the spread of
            # sigma between runs the chains of one run already show
            per_chain = ctx.chain_hist(0).astype(np.int64)
            size = chains // blocks
            rec["blocks"] = []
            for b in range(blocks):
                cnt = per_chain[b * size:(b + 1) * size].sum(axis=0)
                try:
                    rb = pm.equal_height(POTTS, L, lnW, cnt, BETA0 - rec["bracket_half_width"],
                                         BETA0 + rec["bracket_half_width"])
                    rec["blocks"].append({"beta_eqh": rb["beta"], "sigma_od": rb["sigma"],
                                          "k_peaks": list(rb["k_peaks"]), "ln_ratio": rb["sigma"] * 2 * L})
                except pm.MucaError as e:
                    rec["blocks"].append({"error": str(e)})
        return rec, res["lnP"], lnW


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", default="8,16,24,32")
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=2000, help="sweeps per weight iteration")
    ap.add_argument("--cap", type=int, default=150, help="iteration cap per size")
    ap.add_argument("--refine", type=int, default=3)
    ap.add_argument("--therm", type=int, default=2000)
    ap.add_argument("--prod", type=int, default=20000)
    ap.add_argument("--params", default="", help="learned network parameters (mlp_params.npy) for the seed")
    ap.add_argument("--seed-weights", default="",
                    help="log_weights.npz of an earlier run: seed the first size from its largest smaller L")
    ap.add_argument("--weights", default="",
                    help="log_weights.npz of an earlier run: a size with an entry (L<size>) starts from those weights")
    ap.add_argument("--flat-rule", type=int, default=0, choices=[0, 1],
                    help="0: every reachable bin visited and min/max >= 0.5; 1: the paper's [<H>/2, 2<H>]")
    ap.add_argument("--chain-seed", action="store_true",
                    help="seed each size after the first with the previous size's weights, rescaled per site")
    ap.add_argument("--fit-min-l", type=int, default=16, help="smallest L in the 1/L fit")
    ap.add_argument("--max-seconds", type=float, default=600.0, help="wall-time limit of one size's iteration")
    ap.add_argument("--no-iterate", action="store_true",
                    help="with --weights: production on the given weights without iterating them first")
    ap.add_argument("--blocks", type=int, default=0, help="also analyse this many disjoint blocks of chains")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    os.makedirs(args.out, exist_ok=True)
    mlp = None
    if args.params:
        mlp = pm.Mlp(max_samples=1 << 16, seed=1)   # prediction capacity: up to 65536 bins
        mlp.set_params(np.load(args.params))
    results, hists, weights = [], {}, {}
    prev = None
    sizes = [int(x) for x in args.sizes.split(",")]
    if args.seed_weights:
        saved = np.load(args.seed_weights)
        smaller = sorted(int(k[1:]) for k in saved.files if int(k[1:]) < sizes[0])
        if not smaller:
            raise SystemExit(f"{args.seed_weights} holds no size below L={sizes[0]}")
        prev = (smaller[-1], saved[f"L{smaller[-1]}"])
    own = np.load(args.weights) if args.weights else None
    for L in sizes:
        use_prev = prev is not None and (args.chain_seed or (args.seed_weights and L == sizes[0]))
        seed_lnw = rescaled_weights(prev[1], prev[0], L) if use_prev else None
        if own is not None and f"L{L}" in own.files:
            seed_lnw = np.asarray(own[f"L{L}"], np.float64)
        rec, lnP, lnW = run_size(L, args.chains, args.seed, args.sweeps, args.cap, args.refine, args.therm,
                                 args.prod, mlp, args.max_seconds, seed_lnw, args.flat_rule,
                                 iterate=not (args.no_iterate and seed_lnw is not None), blocks=args.blocks)
        results.append(rec)
        if lnP is not None:
            hists[f"L{L}"] = lnP
        if lnW is not None:
            weights[f"L{L}"] = lnW
            prev = (L, lnW)
        print(json.dumps(rec), flush=True)
        with open(os.path.join(args.out, "interface_tension.json"), "w") as fh:
            json.dump({"beta0": BETA0, "runs": results}, fh, indent=1)
        np.savez(os.path.join(args.out, "reweighted_histograms.npz"), **hists)
        np.savez(os.path.join(args.out, "log_weights.npz"), **weights)
    good = [r for r in results if "sigma_od" in r and r["L"] >= args.fit_min_l]
    summary = {"beta0": BETA0, "runs": results}
    if len(good) >= 2:
        s_inf, a = fit_inverse_l([r["L"] for r in good], [r["sigma_od"] for r in good])
        summary["fit"] = {"form": "sigma_inf + a/L", "sizes": [r["L"] for r in good], "sigma_inf": s_inf, "a": a}
        print(json.dumps(summary["fit"]), flush=True)
    with open(os.path.join(args.out, "interface_tension.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    if mlp is not None:
        mlp.close()


if __name__ == "__main__":
    main()
