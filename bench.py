"""Benchmark: spin-update throughput of the multicanonical weight iteration.

One step is one weight iteration: every chain runs the iteration's recorded
sweeps (the sweep kernel), the per-chain histograms are merged, the
recursion lnW <- lnW - ln H is applied and the acceptance tables are
rebuilt.  The default workload is 2D Ising L = 64 with 4096 chains and 2000
sweeps per iteration; --workload potts32 (8-state Potts L = 32, 4096 chains,
5000 sweeps), --workload mixed (nine problems of 512 chains in one launch,
2000 sweeps), mag32 (multimagnetic Ising L = 32) and ising96, ising128,
potts48 (8192 chains, the learned-initial-weights test sizes) measure the
other configurations.  Inputs (spins, tables) are
resident in HBM before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                  [--workload ising64|potts32|mixed|mag32|ising96|ising128|potts48]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-update attempts/s (G/s) + %roofline; sweeps-to-flat, learned vs plain"

# Integer lane operations one Ising update needs by the algorithm (not by
# this kernel's instruction count): a quarter of a Philox4x32-10 block
# (10 rounds x (2 low + 2 high products + 4 xors) = 80 ops / 4 sites = 20)
# plus the update itself (4 neighbour compares, 3 adds, 2 for the table
# index, 1 compare, 2 for the accepted state) = 12.
OPS_PER_ISING_UPDATE = 32
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one int32 op per lane per cycle.
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9
CLOCK_HZ = 2.4e9
OPS_DERIVATION = {
    "ising": "Philox4x32-10: 10 rounds x (2 mul_lo + 2 mul_hi + 4 xor) = 80 lane ops per block of four words, "
             "20 per update; the update: 4 neighbour compares, 3 adds, 2 table-index ops, 1 compare, 2 state ops "
             "= 12; 32 in all.  An estimate that also counts the lane selects of the update (16 ops) gives 36 and "
             "a fraction 1.125 times this one",
    "potts": "half a Philox block (40) + 8 neighbour compares, 6 adds, proposal 3, table index 2, compare 1, "
             "state 2 = 62",
}
# A chain's updates form one dependence chain: each acceptance compare reads
# a threshold that the previous update's outcome selects.  With one chain per
# lane, the compare result read as a lane mask (about 13 cycles on gfx950)
# plus the select (4 cycles) bound a chain to one update per 17 cycles.
DECISION_CHAIN_CYCLES = 17
# One wave per SIMD: 256 CUs x 4 SIMDs x 64 lanes.
LANE_SLOTS = 256 * 4 * 64


def code_text(src: str) -> str:
    """C++ source without comments and with whitespace collapsed, so that a
    change of comments alone leaves the hash below unchanged."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash(root: str = ROOT) -> str:
    """Hash of the sweep kernel's code (comments excluded)."""
    h = hashlib.sha256()
    for f in ("muca_kernels.hip", "muca_device.h"):
        with open(os.path.join(root, "paper_1212_3975_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(updates_per_launch: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "sweep_ising64_c4096_pmc.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_update = d.get("hbm_bytes_per_update")
    return None if per_update is None else per_update * updates_per_launch


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def host_cores():
    """(cores this process may run on, cores the machine reports)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return usable, os.cpu_count() or 1


def cpu_baseline(prob, sweeps: int, n_chains: int, single_chains: int):
    """The oracle as it stands, on the host cores, on a bounded sample of the
    same workload: n_chains chains for `sweeps` sweeps on every thread the
    oracle uses, then single_chains chains on one thread."""
    import oracle

    def run(chains, threads):
        orc = oracle.OracleRun(prob.model, prob.L, chains, prob.seed, q=prob.q, n_threads=threads,
                               beta=getattr(prob, "beta", 0.0))
        t0 = time.perf_counter()
        orc.sweeps(sweeps, oracle.REC_MUCA)
        dt = time.perf_counter() - t0
        return chains * sweeps * prob.N / dt, dt

    threads = oracle.default_threads()
    usable, reported = host_cores()
    ups, dt = run(n_chains, threads)
    ups1, dt1 = run(single_chains, 1)
    name = ["Ising", str(prob.q) + "-state Potts", "multimagnetic Ising"][prob.model]
    return {"value": round(ups / 1e9, 4), "unit": "G/s", "cores": threads, "kind": "oracle",
            "sample": f"{host_cpu_model()}, {threads} threads (the process may use {usable} of the {reported} "
                      f"cores the machine reports; one GPU's share of the host is 16): {n_chains} chains x "
                      f"{sweeps} recorded sweeps of {name} L={prob.L} ({n_chains * sweeps * prob.N:.3g} updates, "
                      f"{dt:.1f} s)",
            "single_core": {"value": round(ups1 / 1e9, 4), "unit": "G/s", "cores": 1,
                            "sample": f"{single_chains} chains x {sweeps} sweeps on one thread "
                                      f"({single_chains * sweeps * prob.N:.3g} updates, {dt1:.1f} s)"},
            "nproc": reported, "usable_cores": usable}


OPS_PER_POTTS_UPDATE = 62   # half a Philox block, the proposal and twice the compares


def scan_chains(L, pm, torch, Problem, model):
    """Sweep-kernel throughput of Ising or 8-state Potts L x L versus the
    number of chains (tuned launch per count): the walkers are serial per
    chain, so throughput grows with the chain count until the chip's LDS holds
    no more walkers."""
    from workloads import POTTS
    potts = model == POTTS
    ops = OPS_PER_POTTS_UPDATE if potts else OPS_PER_ISING_UPDATE
    rows = []
    for chains in (1024, 2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144):
        prob = Problem(model, L, chains, 7, q=8) if potts else Problem(model, L, chains, 7)
        ctx = pm.Muca([prob], device="cuda:0", production=0)
        sweeps = max(20, int(4e9 / (chains * L * L)))
        ctx.sweep(sweeps, pm.REC_NONE)   # warm-up
        ctx.sweep_timing()
        ctx.sweep(sweeps, pm.REC_NONE)
        ms, _ = ctx.sweep_timing()
        rate = chains * L * L * sweeps / (ms * 1e-3)
        info = ctx.launch_info()
        ctx.close()
        rows.append({"chains": chains, "sweeps": sweeps, "kernel_ms": round(ms, 3), "Gups": round(rate / 1e9, 2),
                     "alu_frac": round(ops * rate / PEAK_INT32_OPS, 4),
                     "chains_per_wg": info["chains_per_wg"], "fast_walker": info["fast_walker"],
                     "walker": info["walker"],
                     "workgroups": info["n_workgroups"]})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    name = f"2D 8-state Potts L={L}" if potts else f"2D Ising L={L}"
    print(json.dumps({"metric": "sweep-kernel spin-update attempts/s vs chains", "unit": "G/s",
                      "workload": name, "ops_per_update": ops, "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rng-mode", type=int, default=0)
    ap.add_argument("--chains-per-wg", type=int, default=0)
    ap.add_argument("--fixed", action="store_true",
                    help="skip tuning: 4 helper waves, LDS placement, --chains-per-wg chains per workgroup "
                         "(default 16)")
    ap.add_argument("--no-extra", action="store_true", help="skip the production and reweighting leg")
    ap.add_argument("--workload", default="ising64",
                    choices=["ising64", "potts32", "mixed", "mag32", "ising96", "ising128", "potts48"])
    ap.add_argument("--graph", action="store_true", help="run each iteration as one HIP graph launch")
    ap.add_argument("--scan-chains", type=int, default=0, metavar="L",
                    help="instead of the benchmark: sweep throughput of an L x L lattice versus the number of chains")
    ap.add_argument("--scan-model", default="ising", choices=["ising", "potts8"],
                    help="model of --scan-chains")
    ap.add_argument("--chains", type=int, default=0,
                    help="run a single-problem workload with this many chains instead of its own count "
                         "(a profiling aid; the benchmark line then names the count)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size kernel for "
                         "calibrating rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): runs over several GPUs, which would "
              "shard by chains with one histogram all-reduce per iteration, are not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1212_3975_amd as pm
    from workloads import C2, C3, C4, C_MAG, ISING, Problem

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU: none is visible to this process.", file=sys.stderr)
        sys.exit(2)
    if args.scan_chains:
        from workloads import POTTS
        scan_chains(args.scan_chains, pm, torch, Problem, POTTS if args.scan_model == "potts8" else ISING)
        return

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload in ("ising96", "ising128", "potts48"):
        # the learned-initial-weights test sizes: 8192 chains, 2000 sweeps per iteration
        from workloads import C5_TEST_CHAINS, POTTS
        L = int(args.workload[-3:] if args.workload.endswith("128") else args.workload[-2:])
        model = POTTS if args.workload.startswith("potts") else ISING
        probs = [Problem(model, L, C5_TEST_CHAINS, 1, q=(8 if model == POTTS else 2))]
        M = 2000
    else:
        plan = {"ising64": C2, "potts32": C3, "mixed": C4, "mag32": C_MAG}[args.workload]
        probs = list(plan.problems)
        M = plan.sweeps_per_iter
    if args.chains:
        if len(probs) != 1:
            print("--chains applies to single-problem workloads", file=sys.stderr)
            sys.exit(2)
        p0 = probs[0]
        probs = [Problem(p0.model, p0.L, args.chains, p0.seed, q=p0.q, beta=p0.beta)]
    prob = probs[0]
    torch.cuda.set_device(0)
    opts = dict(rng_mode=args.rng_mode, chains_per_wg=args.chains_per_wg, use_graph=int(args.graph))
    if args.fixed:
        opts.update(rng_mode=5, chains_per_wg=args.chains_per_wg or 16, spin_placement=1, table_placement=1)
    ctx = pm.Muca(probs, device="cuda:0", **opts)
    launch = [ctx.launch_info(i) for i in range(len(probs))]
    updates_per_step = sum(p.n_chains * p.N for p in probs) * M
    single_model = len(probs) == 1
    potts_model = single_model and prob.model == 1
    # algorithmic ops of one step: each problem's updates at its own count
    ops_per_step = sum((OPS_PER_POTTS_UPDATE if p.model == 1 else OPS_PER_ISING_UPDATE) * p.n_chains * p.N
                       for p in probs) * M
    ops_per_update = ops_per_step // updates_per_step if single_model else round(ops_per_step / updates_per_step, 3)

    def step():
        if args.graph:
            return ctx.iterate(M)
        ctx.sweep(M, pm.REC_MUCA)
        return ctx.merge_update(True)

    for _ in range(args.warmup):
        step()
    ctx.sweep_timing()   # reset kernel timing to the timed region

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        stats = step()[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    avg_ms, n_launch = ctx.sweep_timing()

    value = updates_per_step * args.steps / dt / 1e9
    kernel_rate = updates_per_step / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    achieved = ops_per_step / (avg_ms * 1e-3) if avg_ms > 0 else 0.0

    extra = {}
    if not args.no_extra and args.workload == "ising64":
        # production and reweighting leg (reported, not part of the value)
        ctx.clear_production()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        ctx.sweep(200, pm.REC_PROD)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        tr = time.perf_counter()
        ctx.reweight(0, C2.betas)
        tr = time.perf_counter() - tr
        extra = {"production_Gups": round(prob.n_chains * prob.N * 200 / tp / 1e9, 3),
                 "reweight_ms_200_betas": round(tr * 1e3, 3)}
    workload_text = {
        "ising64": "2D Ising L=64 periodic, 4096 chains, one weight iteration of 2000 sweeps "
                   "(sweep + merge + recursion + tables)",
        "potts32": "2D 8-state Potts L=32 periodic, 4096 chains, one weight iteration of 5000 sweeps "
                   "(sweep + merge + recursion + tables)",
        "mixed": "Ising L in {16,24,32,48,64} and 8-Potts L in {8,16,24,32}, 512 chains each, one launch, "
                 "one weight iteration of 2000 sweeps",
        "mag32": "multimagnetic 2D Ising L=32 at beta = 1.5 beta_0 (weights over M), 4096 chains, one weight "
                 "iteration of 2000 sweeps (sweep + merge + recursion + tables)",
        "ising96": "2D Ising L=96 periodic, 8192 chains, one weight iteration of 2000 sweeps from lnW = 0",
        "ising128": "2D Ising L=128 periodic, 8192 chains, one weight iteration of 2000 sweeps from lnW = 0",
        "potts48": "2D 8-state Potts L=48 periodic, 8192 chains, one weight iteration of 2000 sweeps from lnW = 0",
    }[args.workload]
    if args.chains:
        workload_text += f"; run with {args.chains} chains instead"
    # one lane per chain, sequential updates within a chain
    chains = sum(p.n_chains for p in probs)
    bound_ups = chains * CLOCK_HZ / DECISION_CHAIN_CYCLES
    serial = None
    if ops_per_update:
        serial = {"chains": chains, "lane_slots": LANE_SLOTS,
                  "walker_cycles_per_update": round(chains * CLOCK_HZ / (kernel_rate * 1e9), 1),
                  "decision_chain_Gups": round(bound_ups / 1e9, 1),
                  "decision_chain_frac": round(min(1.0, bound_ups * ops_per_update / PEAK_INT32_OPS), 4),
                  "note": f"{chains} chains fill {chains}/{LANE_SLOTS} lane slots; a chain's updates are sequential "
                          f"and each compare reads a threshold selected by the previous outcome (lane-mask read "
                          f"about 13 cycles + select 4), so {chains} chains cannot exceed {chains} x "
                          f"{CLOCK_HZ / 1e9} GHz / {DECISION_CHAIN_CYCLES} cycles with this form; the walker spends "
                          f"walker_cycles_per_update on each (its instruction issue plus LDS waits)"}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "G/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload_text, "problems": [(p.model, p.L, p.n_chains, p.seed) for p in probs],
                   "sweeps_per_iter": M, "graph": bool(args.graph), "launch": launch},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(PEAK_INT32_OPS / 1e12, 2),
                     "unit": "Tops/s (int32 lane ops)", "frac": round(achieved / PEAK_INT32_OPS, 5),
                     "traffic": measured_traffic(updates_per_step) if args.workload == "ising64" else None,
                     "kernel": "sweep_kernel", "kernel_avg_ms": round(avg_ms, 3), "kernel_launches": n_launch,
                     "kernel_rate_Gups": round(kernel_rate, 3), "ops_per_update": ops_per_update,
                     "ops_derivation": OPS_DERIVATION["potts" if potts_model else "ising"] if single_model else
                     "each problem at its own count (Ising and multimagnetic 32, 8-Potts 62), averaged over the "
                     "batch's updates",
                     "serial_chain": serial},
        "extra": dict(extra, last_iter={k: stats[k] for k in ("k_lo", "k_hi", "visited", "reachable", "flat")},
                      kernel_source_hash=kernel_source_hash()),
    }
    ctx.close()
    if not args.no_cpu:
        # about 10-15 s of the oracle on 16 host threads, then about 8 s on one
        big = prob.model != 1
        out["cpu_baseline"] = cpu_baseline(prob, 2000, 2048 if big else 4096, 96 if big else 192)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
