"""Learned initial weights versus the plain recursion: sweeps to a flat histogram.

Orchestration only (every step runs in libmuca.so):

  train   For each training size, iterate the plain recursion from lnW = 0 until
          the merged histogram is flat (every reachable bin visited, min/max >=
          0.5), refine a few more iterations, and add the converged weights to
          the network's training set (ln Omega / N per reachable bin).  Train the
          MLP on the GPU and save its parameters.
  test    For each test size and seed, run both arms with the same seeds: the
          plain recursion from lnW = 0, and the recursion started from the
          network's prediction.  Report the first iteration whose histogram is
          flat, and the sweeps that took per chain and in total.

  python -m paper_1212_3975_amd.learned_init train --out DIR
  python -m paper_1212_3975_amd.learned_init test --params DIR/mlp_params.npy --out DIR
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1212_3975_amd as pm  # noqa: E402
from workloads import C5_SEEDS, C5_TRAIN, ISING, POTTS, Problem  # noqa: E402

NAMES = {ISING: "ising", POTTS: "potts8"}


def iterate_to_flat(ctx, sweeps: int, cap: int, label: str, log_every: int = 10, max_seconds: float = 1e9):
    """Iterates until the merged histogram is flat; returns (first flat
    iteration or None, per-iteration statistics).  Stops at `cap` iterations
    or after `max_seconds` of wall time."""
    hist = []
    t0 = time.time()
    t_log = t0
    for it in range(1, cap + 1):
        if time.time() - t0 > max_seconds:
            print(f"  {label} stopped after {it - 1} iterations ({max_seconds:.0f} s limit)", flush=True)
            break
        st = ctx.iterate(sweeps)[0]
        hist.append({"it": it, "visited": st["visited"], "reachable": st["reachable"],
                     "min_over_max": round(st["min_over_max"], 4), "flat": st["flat"]})
        # a line every log_every iterations, and at least every 30 s on large lattices
        if it % log_every == 0 or st["flat"] or time.time() - t_log > 30.0:
            t_log = time.time()
            print(f"  {label} it={it} visited={st['visited']}/{st['reachable']} "
                  f"min/max={st['min_over_max']:.3f} flat={st['flat']} t={time.time() - t0:.1f}s", flush=True)
        if st["flat"]:
            return it, hist
    return None, hist


def train(out_dir: str, chains: int, sweeps_ising: int, sweeps_potts: int, cap: int, refine: int, steps: int,
          max_seconds: float):
    if steps < 3:
        raise ValueError("steps must be at least 3 (three learning-rate stages)")
    os.makedirs(out_dir, exist_ok=True)
    mlp = pm.Mlp(max_samples=1 << 15, seed=1)
    runs = []
    for i, (model, L) in enumerate(C5_TRAIN):
        prob = Problem(model, L, chains, 1000 + i, q=(2 if model == ISING else 8))
        M = sweeps_ising if model == ISING else sweeps_potts
        print(f"train size {NAMES[model]} L={L} chains={chains} M={M}", flush=True)
        t0 = time.time()
        with pm.Muca([prob]) as ctx:
            n_flat, _ = iterate_to_flat(ctx, M, cap, f"{NAMES[model]}{L}", max_seconds=max_seconds)
            for _ in range(refine if n_flat else 0):
                ctx.iterate(M)
            if n_flat:
                mlp.add_weights(ctx, 0)
        runs.append({"model": NAMES[model], "L": L, "chains": chains, "sweeps_per_iter": M,
                     "iterations_to_flat": n_flat, "seconds": round(time.time() - t0, 2)})
    n = mlp.num_samples()
    print(f"training set: {n} samples", flush=True)
    losses = []
    for lr, k in ((3e-3, steps // 3), (1e-3, steps // 3), (3e-4, steps - 2 * (steps // 3))):
        losses.append(mlp.train(k, lr))
        print(f"  lr={lr} final loss={losses[-1][-1]:.3e}", flush=True)
    params = mlp.params()
    np.save(os.path.join(out_dir, "mlp_params.npy"), params)
    loss = np.concatenate(losses)
    summary = {"runs": runs, "samples": n, "steps": int(loss.size),
               "loss_first": float(loss[0]), "loss_last": float(loss[-1]),
               "rmse_ln_omega_per_site": float(np.sqrt(loss[-1]))}
    with open(os.path.join(out_dir, "train_summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary), flush=True)
    mlp.close()


def test(params_path: str, out_dir: str, sizes, chains: int, sweeps: int, cap_plain: int, cap_learned: int,
         seeds, arms, max_seconds: float = 1e9):
    os.makedirs(out_dir, exist_ok=True)
    mlp = pm.Mlp(max_samples=1 << 16, seed=1)
    mlp.set_params(np.load(params_path))
    results = []
    for model, L in sizes:
        for seed in seeds:
            for arm in arms:
                prob = Problem(model, L, chains, seed, q=(2 if model == ISING else 8))
                label = f"{NAMES[model]}{L} seed={seed} {arm}"
                print(label, flush=True)
                t0 = time.time()
                # arms: "plain" / "learned" start from lnW = 0 / the prediction; a
                # "+corr" suffix turns on the correction function of the recursion
                base, _, extra = arm.partition("+")
                mods = set(extra.split("+")) if extra else set()
                with pm.Muca([prob], correction=int("corr" in mods), update_norm=int("norm" in mods)) as ctx:
                    if base == "learned":
                        mlp.set_log_weights(ctx, 0)
                    cap = cap_learned if base == "learned" else cap_plain
                    n_flat, hist = iterate_to_flat(ctx, sweeps, cap, label, log_every=25, max_seconds=max_seconds)
                iters = n_flat if n_flat else len(hist)   # iterations run (cap or time limit)
                rec = {"model": NAMES[model], "L": L, "seed": seed, "arm": arm, "chains": chains,
                       "sweeps_per_iter": sweeps, "flat": n_flat is not None, "iterations": iters,
                       "sweeps_per_chain": iters * sweeps, "total_sweeps": iters * sweeps * chains,
                       "seconds": round(time.time() - t0, 2),
                       "last_visited": hist[-1]["visited"] if hist else None,
                       "reachable": hist[-1]["reachable"] if hist else None}
                results.append(rec)
                print(json.dumps(rec), flush=True)
                with open(os.path.join(out_dir, "test_results.json"), "w") as fh:
                    json.dump(results, fh, indent=1)
    mlp.close()
    return results


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--out", required=True)
    a.add_argument("--chains", type=int, default=4096)
    a.add_argument("--sweeps-ising", type=int, default=1000)
    a.add_argument("--sweeps-potts", type=int, default=2000)
    a.add_argument("--cap", type=int, default=600)
    a.add_argument("--refine", type=int, default=3)
    a.add_argument("--steps", type=int, default=12000)
    a.add_argument("--max-seconds", type=float, default=150.0, help="wall-time limit per training size")
    b = sub.add_parser("test")
    b.add_argument("--params", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--sizes", default="ising:64,potts8:32")
    b.add_argument("--chains", type=int, default=4096)
    b.add_argument("--sweeps", type=int, default=2000)
    b.add_argument("--cap-plain", type=int, default=400)
    b.add_argument("--cap-learned", type=int, default=100)
    b.add_argument("--seeds", default=",".join(str(s) for s in C5_SEEDS))
    b.add_argument("--arms", default="learned,plain")
    b.add_argument("--max-seconds", type=float, default=1e9, help="wall-time limit per run")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.cmd == "train":
        train(args.out, args.chains, args.sweeps_ising, args.sweeps_potts, args.cap, args.refine, args.steps,
              args.max_seconds)
    else:
        sizes = []
        for tok in args.sizes.split(","):
            name, L = tok.split(":")
            sizes.append((ISING if name == "ising" else POTTS, int(L)))
        test(args.params, args.out, sizes, args.chains, args.sweeps, args.cap_plain, args.cap_learned,
             [int(s) for s in args.seeds.split(",")], args.arms.split(","), args.max_seconds)


if __name__ == "__main__":
    main()
