"""Production runs of the benchmark configurations and the quality of their
reweighted observables (Sec. 5: the specific heat against the exact result,
Eq. 8's mean relative deviation).

  python -m paper_1212_3975_amd.quality --config c2 [--correction] [--out FILE]
  python -m paper_1212_3975_amd.quality --config c3 [--out FILE]

c2 (2D Ising L = 64, 4096 chains): weight iterations of 2000 sweeps (30 of
them as configured, or with the correction function of Sec. 3 until the
histogram is flat), 2000 unrecorded sweeps, 1e5 production sweeps (one
measurement per chain per sweep), then Eq. (2) at 200 beta in [0.3, 0.6].
The statistical error comes from 16 blocks of 256 chains, each reweighted on
its own (mucaReweightStatic on the block's merged counts).
c3 (8-state Potts L = 32, 4096 chains): 50 iterations of 5000 sweeps; the
per-iteration statistics are the result.

Every step runs in the library; this module only sequences the calls and
writes the JSON that the design doc's tables and a CPU test read.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_BLOCKS = 16


def _stats(st):
    return {k: st[k] for k in ("k_lo", "k_hi", "visited", "reachable", "covered", "flat", "min_over_max", "total")}


def run_iterations(ctx, sweeps, n_iters, until_flat, log):
    out = []
    for it in range(n_iters):
        st = ctx.iterate(sweeps)[0]
        out.append(_stats(st))
        print(f"  iteration {it + 1}: k {st['k_lo']}..{st['k_hi']}, visited {st['visited']}/{st['reachable']}, "
              f"min/max {st['min_over_max']:.3f}, flat {st['flat']}", file=log, flush=True)
        if until_flat and st["flat"]:
            break
    return out


def production(pm, ctx, prob, n_therm, n_prod, betas, log, chunk=10_000):
    """Thermalisation, production in launches of `chunk` sweeps, Eq. (2) on
    the whole production and on N_BLOCKS blocks of chains."""
    ctx.sweep(n_therm, pm.REC_NONE)
    ctx.clear_production()
    t0 = time.perf_counter()
    done = 0
    while done < n_prod:
        n = min(chunk, n_prod - done)
        ctx.sweep(n, pm.REC_PROD)
        done += n
        ctx.sweep_timing()
        print(f"  production {done}/{n_prod} sweeps", file=log, flush=True)
    prod_s = time.perf_counter() - t0
    e, c, m = ctx.reweight(0, betas)
    cnt = ctx.prod_counts()
    lnW = ctx.lnW()
    per_chain = ctx.chain_hist().astype(np.int64)   # production counts per chain, [C][bins]
    blocks = []
    size = prob.n_chains // N_BLOCKS
    for b in range(N_BLOCKS):
        cb = per_chain[b * size:(b + 1) * size].sum(axis=0)
        eb, cvb, _ = pm.reweight_static(prob.model, prob.L, lnW, cb, np.zeros_like(cb), betas)
        blocks.append({"e": eb.tolist(), "c_v": cvb.tolist()})
    nz = np.flatnonzero(cnt)
    return {"n_therm": n_therm, "n_prod": n_prod, "production_s": round(prod_s, 2),
            "counts_k_lo": int(nz[0]), "counts_k_hi": int(nz[-1]), "bins_with_data": int(nz.size),
            "betas": list(map(float, betas)), "e": e.tolist(), "c_v": c.tolist(), "abs_m": m.tolist(),
            "blocks": blocks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=["c2", "c3"], required=True)
    ap.add_argument("--correction", action="store_true", help="correction function; iterate until flat")
    ap.add_argument("--max-iters", type=int, default=100)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    import torch
    import paper_1212_3975_amd as pm
    from workloads import C2, C3

    if not torch.cuda.is_available():
        print("needs a GPU", file=sys.stderr)
        sys.exit(2)
    plan = C2 if args.config == "c2" else C3
    prob = plan.problems[0]
    log = sys.stderr
    res = {"config": args.config, "problem": [prob.model, prob.L, prob.n_chains, prob.seed, prob.q],
           "correction": bool(args.correction), "sweeps_per_iter": plan.sweeps_per_iter}
    with pm.Muca([prob], correction=int(args.correction)) as ctx:
        res["launch"] = ctx.launch_info()
        t0 = time.perf_counter()
        n = args.max_iters if args.correction else plan.n_iters
        res["iterations"] = run_iterations(ctx, plan.sweeps_per_iter, n, args.correction, log)
        res["iterations_s"] = round(time.perf_counter() - t0, 2)
        if args.config == "c2":
            res["production"] = production(pm, ctx, prob, plan.n_therm, plan.n_prod, np.array(plan.betas), log)
        res["lnW"] = ctx.lnW().tolist()
    out = args.out or os.path.join(ROOT, "results", "quality",
                                   f"{args.config}{'_corr' if args.correction else ''}.json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        json.dump(res, fh)
    print(json.dumps({k: v for k, v in res.items() if k not in ("iterations", "production", "lnW")}), flush=True)


if __name__ == "__main__":
    main()
