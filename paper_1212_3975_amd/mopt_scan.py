"""Optimal sweeps per iteration and chain (Sec. 4, Figs. 2-3 and 6) at GPU chain counts.

Orchestration only (every step runs in libmuca.so).  For each model, lattice
size L, number of chains p, sweeps per iteration M and seed:
  1. Start from lnW = 0 at infinite temperature.
  2. Iterate the recursion, with the correction function and the paper's
     convergence rule (every entry within [<H>/2, 2<H>]), until the first
     flat histogram.
  3. Record N_iter.
Per (L, p), the total statistics N_iter M p averaged over the seeds is
minimal at M~_opt(p).  The paper fits M_opt(L, p) = M_1(L) / p; Eq. (5)
gives M_1 = 5.7 L^2.51 (Ising) and 24 L^2.67 (8-state Potts).  This driver
fits M_1 over the chain counts and reports where the 1/p law stops holding.

The scan over M runs from the largest M down.  One run may spend at most
--max-total chain-sweeps (and --cap iterations); a run that reaches either
limit has not converged.  The scan of a p stops at the first M where a seed
does not converge (except for a run cut by the work limit before any M has
converged: smaller M get more iterations), or where a seed alone spends more than seeds x the best
mean so far (the mean at that M then exceeds the best), or where the mean
exceeds twice the best: the total statistics is taken to rise monotonically
below its minimum.  An optimum at the largest M scanned is flagged
"upper_edge": the minimum may lie above the scanned range.
The models are Ising, 8-state Potts, and the multimagnetic Ising ensemble at
beta = (3/2) beta_0, whose weights are over the magnetization.

  python -m paper_1212_3975_amd.mopt_scan --model mag --sizes 8,16 --out DIR
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
from workloads import ISING, ISING_MAG, POTTS, Problem  # noqa: E402

BETA0_ISING = 0.5 * math.log(1.0 + math.sqrt(2.0))   # Sec. 3
MODELS = {"ising": ISING, "potts8": POTTS, "mag": ISING_MAG}
EQ5 = {"ising": (5.7, 0.51), "potts8": (24.0, 0.67)}   # Eq. (5): M_1 = a L^(2 + b)


def problem(model_name, L, p, seed):
    if model_name == "potts8":
        return Problem(POTTS, L, p, seed, q=8)
    if model_name == "mag":
        return Problem(ISING_MAG, L, p, seed, beta=1.5 * BETA0_ISING)
    return Problem(ISING, L, p, seed)


def iterations_to_flat(model_name, L, p, M, seed, cap, launch):
    with pm.Muca([problem(model_name, L, p, seed)], correction=1, flat_rule=1, production=0, **launch) as ctx:
        for it in range(1, cap + 1):
            if ctx.iterate(M)[0]["flat"]:
                return it
    return None


def scan_p(model_name, L, p, sweeps, seeds, cap, max_total, launch, log):
    """Descending scan over M at one chain count; returns (best record or
    None, list of records)."""
    best, recs = None, []
    for M in sorted(sweeps, reverse=True):
        work_cap = max_total if best is None else min(max_total, seeds * best["total_sweeps"])
        it_cap = min(cap, int(work_cap // (M * p)))
        if it_cap < 1:
            continue
        its, t0 = [], time.time()
        for s in range(1, seeds + 1):
            its.append(iterations_to_flat(model_name, L, p, M, s, it_cap, launch))
            if its[-1] is None:
                break
        rec = {"L": L, "p": p, "M": M, "n_iter": its, "iteration_cap": it_cap,
               "converged": sum(i is not None for i in its), "seconds": round(time.time() - t0, 2)}
        complete = len(its) == seeds and rec["converged"] == seeds
        if complete:
            rec["mean_n_iter"] = float(np.mean(its))
            rec["total_sweeps"] = rec["mean_n_iter"] * M * p
        recs.append(rec)
        log(rec)
        if not complete:
            # before any M has converged, a run cut by the work cap (not by
            # the iteration cap) says nothing about smaller M, which may
            # spend more iterations
            if best is None and it_cap < cap:
                continue
            break
        if best is None or rec["total_sweeps"] < best["total_sweeps"]:
            best = rec
        elif rec["total_sweeps"] > 2.0 * best["total_sweeps"]:
            break
    if best is not None:
        last = recs[-1]
        # the next M down hit the iteration cap with a work below the best:
        # its mean might still have been lower
        cap_bound = (last is not best and "mean_n_iter" not in last and last["iteration_cap"] == cap
                     and cap * last["M"] * p < best["total_sweeps"])
        best = dict(best, upper_edge=best["M"] == recs[0]["M"], cap_bound=cap_bound)
    return best, recs


def fit_m1(ps, mopts):
    """Least squares of log M_opt = log M_1 - log p (slope fixed at -1)."""
    return float(np.exp(np.mean(np.log(np.asarray(mopts, float)) + np.log(np.asarray(ps, float)))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--model", default="ising", choices=sorted(MODELS))
    ap.add_argument("--sizes", default="8,16")
    ap.add_argument("--chains", default="64,256,1024,4096")
    ap.add_argument("--sweeps", default="1,2,4,8,16,32,64,128,256,512,1024,2048,4096")
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--cap", type=int, default=400, help="iteration cap of one run")
    ap.add_argument("--max-total", type=float, default=4e8,
                    help="work limit of one run, in chain-sweeps (N_iter M p)")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    os.makedirs(args.out, exist_ok=True)
    # fixed launch (no tuning per context): 16 chains per workgroup (small chain
    # counts still spread over several CUs), producer waves, lattice and table
    # in LDS, so that the fast walkers run where they have a compiled shape
    launch = dict(rng_mode=4, chains_per_wg=16, spin_placement=1, table_placement=1)
    sizes = [int(x) for x in args.sizes.split(",")]
    chains = [int(x) for x in args.chains.split(",")]
    sweeps = [int(x) for x in args.sweeps.split(",")]
    runs, summary = [], {"model": args.model, "flat_rule": "[<H>/2, 2<H>] and full range", "correction": True,
                         "beta": 1.5 * BETA0_ISING if args.model == "mag" else None, "sizes": {}}
    t_start = time.time()
    for L in sizes:
        per_p = {}
        for p in chains:
            best, recs = scan_p(args.model, L, p, sweeps, args.seeds, args.cap, args.max_total, launch,
                                lambda r: print(json.dumps(r), flush=True))
            runs.extend(recs)
            if best is not None:
                per_p[p] = {"M_opt": best["M"], "mean_n_iter": best["mean_n_iter"],
                            "total_sweeps": best["total_sweeps"], "upper_edge": best["upper_edge"],
                            "cap_bound": best["cap_bound"]}
            with open(os.path.join(args.out, f"mopt_{args.model}.json"), "w") as fh:
                json.dump({"summary": summary, "runs": runs}, fh, indent=1)
        entry = {"per_p": per_p}
        if len(per_p) >= 2:
            ps = sorted(per_p)
            entry["M1_fit"] = fit_m1(ps, [per_p[q]["M_opt"] for q in ps])
        if args.model in EQ5:
            a, b = EQ5[args.model]
            entry["M1_eq5"] = a * L ** (2 + b)
        summary["sizes"][L] = entry
        print(json.dumps({"L": L, **entry}), flush=True)
    summary["seconds"] = round(time.time() - t_start, 1)
    with open(os.path.join(args.out, f"mopt_{args.model}.json"), "w") as fh:
        json.dump({"summary": summary, "runs": runs}, fh, indent=1)


if __name__ == "__main__":
    main()
