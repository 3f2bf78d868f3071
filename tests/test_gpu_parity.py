"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer state (spins, energies, per-chain and merged histograms), the
log-weights and the acceptance tables must match bit for bit; reweighted
observables to a relative 1e-10.  Runs on an MI355X (marked gpu)."""
import numpy as np
import pytest

import oracle
from conftest import device_table, gpu_available
from workloads import C1, ISING, ISING_MAG, POTTS, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _pm():
    import paper_1212_3975_amd as pm
    return pm


def _orc(prob: Problem, chain0=0, n=None):
    return oracle.OracleRun(prob.model, prob.L, n if n is not None else prob.n_chains, prob.seed, q=prob.q,
                            chain0=chain0, beta=prob.beta)


def _orc_iteration(orc, n_sweeps):
    orc.hist[:] = 0
    orc.sweeps(n_sweeps, oracle.REC_MUCA)
    per_chain = orc.hist.copy()
    H = orc.merged()
    oracle.lib().orc_recursion(orc.n_bins, H, orc.lnW)
    orc.T = orc._table()
    orc.hist[:] = 0
    return per_chain, H


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64), np.asarray(b, np.float64).view(np.uint64))


def _compare_iterations(ctx, orc, n_iters, n_sweeps, prob_idx=0, check_chain_hist=True):
    for it in range(n_iters):
        print(f"  iteration {it}", flush=True)
        if check_chain_hist:
            ctx.sweep(n_sweeps, 1)
            ch = ctx.chain_hist(prob_idx)
            stats = ctx.merge_update(True)[prob_idx]
        else:
            stats = ctx.iterate(n_sweeps)[prob_idx]
        pc, H = _orc_iteration(orc, n_sweeps)
        if check_chain_hist:
            assert np.array_equal(ch, pc), f"per-chain histograms differ at iteration {it}"
        assert np.array_equal(ctx.H(prob_idx), H), f"merged H differs at iteration {it}"
        fl = oracle.flatness(H, orc.mask)
        assert bool(stats["flat"]) == fl.flat and bool(stats["covered"]) == fl.covered
        assert stats["total"] == orc.n_chains * n_sweeps
        assert _same_bits(ctx.lnW(prob_idx), orc.lnW), f"lnW differs at iteration {it}"
        assert np.array_equal(ctx.table(prob_idx), device_table(orc)), f"T differs at iteration {it}"
        assert np.array_equal(ctx.spins(prob_idx), orc.spins), f"spins differ at iteration {it}"
        assert np.array_equal(ctx.k(prob_idx), orc.k), f"k differs at iteration {it}"
        assert np.array_equal(ctx.m(prob_idx), orc.m), f"M differs at iteration {it}"


def test_initial_state_matches():
    pm = _pm()
    for prob in (Problem(ISING, 8, 70, 5), Problem(POTTS, 5, 33, 6, q=8), Problem(ISING, 64, 64, 1)):
        print("case", prob, flush=True)
        with pm.Muca([prob]) as ctx:
            orc = _orc(prob)
            assert np.array_equal(ctx.spins(), orc.spins)
            assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m)
            assert np.array_equal(ctx.reachable(), orc.mask)
            assert np.array_equal(ctx.table(), device_table(orc))


def test_c1_ising_L8_full_run_bit_exact():
    """Ising L = 8, 4 chains, 20 iterations of 1e4 sweeps: every iteration's
    per-chain and merged histograms, weights, tables and spins."""
    pm = _pm()
    prob = C1.problems[0]
    with pm.Muca([prob]) as ctx:
        print("launch", ctx.launch_info(), flush=True)
        orc = _orc(prob)
        _compare_iterations(ctx, orc, C1.n_iters, C1.sweeps_per_iter)


CONFIGS = [dict(rng_mode=1, chains_per_wg=16, spin_placement=1, table_placement=1),
           dict(rng_mode=2, chains_per_wg=32, spin_placement=1, table_placement=2),
           dict(rng_mode=3, chains_per_wg=64, spin_placement=2, table_placement=1),
           dict(rng_mode=4, chains_per_wg=8, spin_placement=2, table_placement=2),
           dict(rng_mode=2, chains_per_wg=4, spin_placement=1, table_placement=1)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "-".join(f"{k[:4]}{v}" for k, v in c.items()))
@pytest.mark.parametrize("prob", [Problem(ISING, 6, 100, 7), Problem(POTTS, 3, 70, 8, q=8),
                                  Problem(POTTS, 7, 41, 9, q=8), Problem(ISING, 12, 65, 10),
                                  Problem(POTTS, 9, 20, 11, q=3), Problem(ISING, 16, 40, 12),
                                  Problem(ISING, 24, 33, 13), Problem(POTTS, 16, 40, 14, q=8),
                                  Problem(POTTS, 24, 21, 15, q=8)],
                         ids=lambda p: f"{'ising' if p.model == 0 else 'potts'}L{p.L}C{p.n_chains}")
def test_launch_configurations_bit_exact(prob, cfg):
    """Ragged chain counts, lattices that end inside a chunk, every random-number
    mode and placement: all give the oracle's trajectories."""
    pm = _pm()
    print("case", prob, cfg, flush=True)
    with pm.Muca([prob], **cfg) as ctx:
        info = ctx.launch_info()
        placed = cfg["rng_mode"] > 1 and cfg["spin_placement"] == 1 and cfg["table_placement"] == 1
        fast_shape = ((prob.model == ISING and prob.L in (16, 24, 32, 48, 64)) or
                      (prob.model == POTTS and prob.q == 8 and prob.L in (16, 24, 32)))
        fast_expected = placed and fast_shape
        assert info["fast_walker"] == int(fast_expected), info
        orc = _orc(prob)
        _compare_iterations(ctx, orc, 4, 150)


def test_batched_problems_match_oracle_and_single_runs():
    """Several problems in one launch: each equals its own oracle run and the
    same problem run alone (batching invariance)."""
    pm = _pm()
    probs = [Problem(ISING, 16, 40, 1), Problem(ISING, 10, 64, 2), Problem(POTTS, 8, 50, 3, q=8),
             Problem(POTTS, 5, 17, 4, q=8)]
    with pm.Muca(probs) as ctx:
        orcs = [_orc(p) for p in probs]
        for it in range(3):
            print(f"  iteration {it}", flush=True)
            ctx.iterate(120)
            for j, o in enumerate(orcs):
                _, H = _orc_iteration(o, 120)
                assert np.array_equal(ctx.H(j), H)
                assert _same_bits(ctx.lnW(j), o.lnW)
                assert np.array_equal(ctx.spins(j), o.spins)
    with pm.Muca([probs[2]]) as alone:
        for it in range(3):
            alone.iterate(120)
        assert np.array_equal(alone.spins(), orcs[2].spins)


def test_graph_iteration_equals_eager():
    pm = _pm()
    prob = Problem(ISING, 16, 96, 12)
    with pm.Muca([prob], use_graph=1) as g, pm.Muca([prob], use_graph=0) as e:
        for it in range(4):
            print(f"  iteration {it}", flush=True)
            sg = g.iterate(300)[0]
            se = e.iterate(300)[0]
            assert sg == se
            assert np.array_equal(g.H(), e.H())
            assert _same_bits(g.lnW(), e.lnW())
            assert np.array_equal(g.spins(), e.spins())
        orc = _orc(prob)
        for _ in range(4):
            _orc_iteration(orc, 300)
        assert np.array_equal(g.spins(), orc.spins) and _same_bits(g.lnW(), orc.lnW)


def test_production_and_reweighting():
    """Production counts and |M| sums bit for bit; Eq. (2) reweighting to
    1e-10 relative on 200 inverse temperatures."""
    pm = _pm()
    for prob in (Problem(ISING, 8, 64, 21), Problem(POTTS, 6, 48, 22, q=8)):
        print("case", prob, flush=True)
        with pm.Muca([prob]) as ctx:
            orc = _orc(prob)
            for _ in range(8):
                ctx.iterate(500)
                _orc_iteration(orc, 500)
            ctx.sweep(300, pm.REC_NONE)
            ctx.clear_production()
            ctx.sweep(2000, pm.REC_PROD)
            cnt, sab = orc.production(300, 2000)
            assert np.array_equal(ctx.prod_counts(), cnt)
            if prob.model == ISING:
                assert np.array_equal(ctx.prod_absm(), sab)
            betas = np.linspace(0.3, 0.6, 200)
            e, c, m = ctx.reweight(0, betas)
            eo, co, mo = oracle.reweight(prob.model, prob.L, orc.lnW, cnt, sab, betas)
            np.testing.assert_allclose(e, eo, rtol=1e-10, atol=0)
            np.testing.assert_allclose(c, co, rtol=1e-10, atol=0)
            if prob.model == ISING:
                np.testing.assert_allclose(m, mo, rtol=1e-10, atol=0)
            else:
                assert np.all(np.isnan(m))


@pytest.mark.parametrize("prob", [Problem(POTTS, 8, 40, 31, q=8), Problem(ISING_MAG, 16, 40, 32, beta=0.66)],
                         ids=["potts", "mag"])
def test_checkpoint_restore_continues_bit_exact(prob):
    pm = _pm()
    with pm.Muca([prob]) as a:
        for _ in range(3):
            a.iterate(200)
        blob = a.checkpoint()
        for _ in range(2):
            a.iterate(200)
        with pm.Muca([prob]) as b:
            b.restore(blob)
            assert b.sweep_count() == 600
            for _ in range(2):
                b.iterate(200)
            assert np.array_equal(a.spins(), b.spins()) and _same_bits(a.lnW(), b.lnW())
            assert np.array_equal(a.H(), b.H())
            assert np.array_equal(a.k(), b.k()) and np.array_equal(a.m(), b.m())
    # a checkpoint of another beta is refused
    if prob.model == ISING_MAG:
        other = Problem(ISING_MAG, prob.L, prob.n_chains, prob.seed, beta=prob.beta + 0.1)
        with pm.Muca([other]) as c:
            with pytest.raises(pm.MucaError, match="differs"):
                c.restore(blob)


def test_set_log_weights_canonical_limit():
    """Weights lnW = -beta E installed through the ABI give canonical
    Metropolis; trajectories equal the oracle's with the same weights."""
    pm = _pm()
    prob = Problem(ISING, 10, 64, 41)
    lnW = -0.44 * oracle.energies(ISING, 10)
    with pm.Muca([prob]) as ctx:
        ctx.set_log_weights(0, lnW)
        orc = _orc(prob)
        orc.set_log_weights(lnW)
        assert np.array_equal(ctx.table(), device_table(orc))
        ctx.sweep(500, pm.REC_MUCA)
        orc.sweeps(500, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        assert np.array_equal(ctx.spins(), orc.spins)


def test_errors_are_reported():
    pm = _pm()
    with pm.Muca([Problem(ISING, 8, 4, 1)], production=0) as ctx:
        with pytest.raises(pm.MucaError):
            ctx.sweep(10, pm.REC_PROD)
        with pytest.raises(pm.MucaError):
            ctx.set_log_weights(0, np.zeros(5))
        with pytest.raises(pm.MucaError):
            ctx.reweight(0, [0.4])
        with pytest.raises(pm.MucaError):
            ctx.set_log_weights(0, np.full(129, np.nan))


@pytest.mark.parametrize("prob", [Problem(ISING, 16, 48, 51), Problem(POTTS, 8, 40, 52, q=8)],
                         ids=["ising16", "potts8"])
def test_correction_function_bit_exact(prob):
    pm = _pm()
    with pm.Muca([prob], correction=1) as ctx:
        orc = _orc(prob)
        for it in range(6):
            print(f"  iteration {it}", flush=True)
            st = ctx.iterate(150)[0]
            H, fl, _ = orc.iterate(150, correct=True)
            assert np.array_equal(ctx.H(), H)
            assert _same_bits(ctx.lnW(), orc.lnW), f"lnW differs at iteration {it}"
            assert np.array_equal(ctx.spins(), orc.spins)


@pytest.mark.parametrize("prob,correct", [(Problem(ISING, 16, 48, 61), False), (Problem(POTTS, 8, 40, 62, q=8), False),
                                          (Problem(ISING, 12, 32, 63), True)],
                         ids=["ising16", "potts8", "ising12-corr"])
def test_normalized_update_bit_exact(prob, correct):
    """The recursion with its update shifted to zero mean over the visited
    bins (update_norm = 1), alone and followed by the correction function:
    weights as bits, histograms and trajectories equal the oracle's over six
    iterations, through mucaIterate."""
    pm = _pm()
    with pm.Muca([prob], update_norm=1, correction=int(correct)) as ctx:
        orc = _orc(prob)
        for it in range(6):
            print(f"  iteration {it}", flush=True)
            ctx.iterate(150)
            H, _, _ = orc.iterate(150, correct=correct, norm=True)
            assert np.array_equal(ctx.H(), H)
            assert _same_bits(ctx.lnW(), orc.lnW), f"lnW differs at iteration {it}"
            assert np.array_equal(ctx.table(), device_table(orc))
            assert np.array_equal(ctx.spins(), orc.spins)


@pytest.mark.parametrize("rule,ratio,want", [(1, 0.5, [0] * 7 + [1] * 5), (0, 0.3, [0] * 6 + [1] * 6),
                                              (0, 0.75, [0] * 9 + [1, 1, 0])],
                         ids=["paper-rule", "ratio0.3", "ratio0.75"])
def test_flatness_options_match_oracle(rule, ratio, want):
    """The library's flatness test with the paper's rule (every reachable
    entry within [avg/2, 2 avg], Sec. 3) and with other min/max thresholds:
    every statistic and decision equals the oracle's on the same merged
    histogram.  The expected decision sequences come from the oracle and
    contain both outcomes."""
    pm = _pm()
    prob = Problem(ISING, 8, 64, 61)
    with pm.Muca([prob], flat_rule=rule, flat_ratio=ratio) as ctx:
        orc = _orc(prob)
        got = []
        for it in range(12):
            print(f"  iteration {it}", flush=True)
            st = ctx.iterate(1000)[0]
            H, fl, _ = orc.iterate(1000, ratio=ratio, rule=rule)
            assert np.array_equal(ctx.H(), H)
            assert (bool(st["flat"]), bool(st["covered"])) == (fl.flat, fl.covered), f"iteration {it}"
            assert (st["k_lo"], st["k_hi"], st["visited"], st["reachable"]) == (fl.k_lo, fl.k_hi, fl.visited,
                                                                                 fl.reachable)
            assert st["total"] == int(H.sum())
            for key in ("min_over_max", "min_over_avg", "max_over_avg"):
                assert st[key] == pytest.approx(getattr(fl, key), rel=1e-14, abs=0.0), key
            got.append(int(fl.flat))
        assert got == want


def test_interface_tension_of_a_production_run():
    """8-state Potts L=16: weights iterated (with the correction function) to a
    flat histogram, a production run, then the equal-height analysis (Sec. 5,
    Eq. 9) of the library on its own production data against the oracle's on
    the same counts and weights."""
    import math
    pm = _pm()
    prob = Problem(POTTS, 16, 2048, 61, q=8)
    b0 = math.log(1.0 + math.sqrt(8.0))
    with pm.Muca([prob], correction=1) as ctx:
        flat = False
        for it in range(150):
            if ctx.iterate(1000)[0]["flat"]:
                flat = True
                break
        assert flat, "no flat histogram within 150 iterations"
        ctx.sweep(1000, pm.REC_NONE)
        ctx.sweep(4000, pm.REC_PROD)
        got = ctx.interface_tension(0, b0 - 0.05, b0 + 0.05)
        cnt, lnW = ctx.prod_counts(0), ctx.lnW(0)
    assert cnt.sum() == 2048 * 4000
    beta, sigma, ks = oracle.interface_tension(POTTS, 16, lnW, cnt, b0 - 0.05, b0 + 0.05)
    print(f"  beta_eqh={got['beta']:.6f} sigma={got['sigma']:.5f} peaks={got['k_peaks']}", flush=True)
    assert got["beta"] == pytest.approx(beta, rel=1e-12)
    assert got["sigma"] == pytest.approx(sigma, rel=1e-10)
    assert got["k_peaks"] == ks
    # a first-order double peak: ordered peak at low k, disordered at high k
    assert ks[0] < ks[1] < ks[2] and 0.0 < got["sigma"] < 0.2



MAG_PROBS = [Problem(ISING_MAG, 6, 100, 21, beta=0.66), Problem(ISING_MAG, 16, 40, 22, beta=0.4407),
             Problem(ISING_MAG, 12, 65, 23, beta=1.1), Problem(ISING_MAG, 24, 33, 24, beta=0.66),
             Problem(ISING_MAG, 32, 20, 25, beta=0.5)]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "-".join(f"{k[:4]}{v}" for k, v in c.items()))
@pytest.mark.parametrize("prob", MAG_PROBS, ids=lambda p: f"mag L{p.L}C{p.n_chains}b{p.beta}")
def test_multimagnetic_bit_exact(prob, cfg):
    """Multimagnetic Ising (weights over M at fixed beta, Sec. 4) in every
    launch configuration, the generic walker and the fast one: spins, k, M,
    per-chain and merged histograms over m, weights and the two-factor tables
    equal the oracle's."""
    pm = _pm()
    print("case", prob, cfg, flush=True)
    with pm.Muca([prob], **cfg) as ctx:
        placed = cfg["rng_mode"] > 1 and cfg["spin_placement"] == 1 and cfg["table_placement"] == 1
        assert ctx.launch_info()["fast_walker"] == int(placed and prob.L in (16, 24, 32, 48, 64))
        orc = _orc(prob)
        assert ctx.table().shape == (prob.L * prob.L + 1, 10)
        assert np.array_equal(ctx.table(), device_table(orc))
        assert np.array_equal(ctx.reachable(), orc.mask)
        _compare_iterations(ctx, orc, 4, 150)


def test_multimagnetic_batched_with_energy_models_and_production():
    """A multimagnetic problem batched with Ising and Potts problems in one
    launch; then production counts and the k sums per m bin."""
    pm = _pm()
    probs = [Problem(ISING_MAG, 8, 48, 31, beta=0.66), Problem(ISING, 8, 40, 32), Problem(POTTS, 6, 24, 33, q=8)]
    with pm.Muca(probs, correction=1) as ctx:
        orcs = [_orc(p) for p in probs]
        for it in range(3):
            print(f"  iteration {it}", flush=True)
            ctx.iterate(200)
            for j, o in enumerate(orcs):
                H, _, _ = o.iterate(200, correct=True)
                assert np.array_equal(ctx.H(j), H)
                assert _same_bits(ctx.lnW(j), o.lnW)
                assert np.array_equal(ctx.spins(j), o.spins)
                assert np.array_equal(ctx.table(j), device_table(o))
        ctx.sweep(100, pm.REC_NONE)
        ctx.sweep(300, pm.REC_PROD)
        cnt, ksum = ctx.prod_counts(0), ctx.prod_absm(0)
        for o in orcs:
            o.sweeps(100, oracle.REC_NONE)
        ocnt, oks = orcs[0].production(0, 300)
        assert np.array_equal(cnt, ocnt) and np.array_equal(ksum, oks)
        with pytest.raises(pm.MucaError, match="weights over E"):
            ctx.reweight(0, [0.3, 0.4])


@pytest.mark.parametrize("L", [16, 48])
def test_multimagnetic_fast_walker_production(L):
    """The fast walker's multimagnetic variant: after weight iterations, a
    production run's counts per m and sums of k per m (k recounted from the
    LDS lattice each sweep) equal the oracle's, and so do the final k and M."""
    pm = _pm()
    prob = Problem(ISING_MAG, L, 40, 26 + L, beta=0.66)
    with pm.Muca([prob], rng_mode=4, chains_per_wg=16, spin_placement=1, table_placement=1) as ctx:
        assert ctx.launch_info()["fast_walker"] == 1
        orc = _orc(prob)
        for it in range(3):
            ctx.iterate(100)
            orc.iterate(100)
        ctx.sweep(50, pm.REC_NONE)
        ctx.sweep(120, pm.REC_PROD)
        orc.sweeps(50, oracle.REC_NONE)
        cnt, ksum = orc.production(0, 120)
        assert np.array_equal(ctx.prod_counts(), cnt) and np.array_equal(ctx.prod_absm(), ksum)
        assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m)
        assert np.array_equal(ctx.spins(), orc.spins)


@pytest.mark.parametrize("chains,cw", [(100, 64), (40, 32)], ids=["c100-cw64", "c40-cw32"])
def test_packed_l64_walker_bit_exact(chains, cw):
    """Ising L = 64 with more than 16 chains per workgroup keeps the lattices as
    bits (the streamed walker on bit lattices; with 32 + 8 chains one launch
    mixes it with the byte walker): trajectories, histograms, weights, and
    production counts and |M| sums equal the oracle's."""
    pm = _pm()
    prob = Problem(ISING, 64, chains, 41 + chains)
    with pm.Muca([prob], rng_mode=4, chains_per_wg=cw, spin_placement=1, table_placement=1) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["fast_walker"] == 1 and info["chains_per_wg"] == cw
        orc = _orc(prob)
        _compare_iterations(ctx, orc, 3, 40)
        ctx.sweep(20, pm.REC_NONE)
        ctx.sweep(30, pm.REC_PROD)
        orc.sweeps(20, oracle.REC_NONE)
        cnt, sab = orc.production(0, 30)
        assert np.array_equal(ctx.prod_counts(), cnt) and np.array_equal(ctx.prod_absm(), sab)
        assert np.array_equal(ctx.spins(), orc.spins)


@pytest.mark.parametrize("rng_mode", [2, 4, 5], ids=["one-producer", "three-producers", "four-producers"])
@pytest.mark.parametrize("prob,n_sweeps,cw", [(Problem(ISING, 16, 40, 51), 3000, 16),
                                              (Problem(POTTS, 16, 40, 52, q=8), 3000, 16),
                                              (Problem(ISING_MAG, 16, 40, 53, beta=0.66), 3000, 16),
                                              (Problem(POTTS, 24, 30, 54, q=8), 1500, 16),
                                              (Problem(POTTS, 32, 60, 57, q=8), 600, 47),
                                              (Problem(POTTS, 16, 80, 58, q=8), 1500, 64),
                                              (Problem(POTTS, 24, 80, 59, q=8), 800, 64),
                                              (Problem(ISING, 64, 20, 55), 600, 16),
                                              (Problem(ISING, 64, 80, 56), 300, 64)],
                         ids=["isingL16", "pottsL16", "magL16", "pottsL24", "pottsL32-wide", "pottsL16-wide",
                              "pottsL24-wide", "isingL64", "isingL64-packed"])
def test_fast_walkers_long_launch_bit_exact(prob, n_sweeps, cw, rng_mode):
    """One long launch of each fast walker with non-trivial weights: thousands
    of chunk hand-offs between the producer waves (which read the lattice one or
    two chunks ahead of the walker) and the walker, with one or three producer
    waves.  L = 16 has four chunks per sweep, the fewest the walkers allow; the
    wide cases run the Potts walker with its small chunks and the Ising L = 64
    walker on bit lattices (each next to a narrow work item for the remaining
    chains).
    Trajectories, per-chain histograms and energies equal the oracle's."""
    pm = _pm()
    print("case", prob, n_sweeps, cw, rng_mode, flush=True)
    with pm.Muca([prob], rng_mode=rng_mode, chains_per_wg=cw, spin_placement=1, table_placement=1) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["fast_walker"] == 1
        orc = _orc(prob)
        _compare_iterations(ctx, orc, 1, 200)   # non-trivial weights
        ctx.sweep(n_sweeps, pm.REC_MUCA)
        orc.hist[:] = 0
        orc.sweeps(n_sweeps, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        assert np.array_equal(ctx.spins(), orc.spins)
        assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m)


@pytest.mark.parametrize("prob,bad", [(Problem(ISING, 8, 16, 71), 2), (Problem(POTTS, 8, 16, 72, q=8), 8)],
                         ids=["ising", "potts8"])
def test_restore_rejects_out_of_range_spins(prob, bad):
    """A checkpoint holding a spin outside 0..q-1 is refused on the host before
    any state changes (no sweep runs on it); the intact blob still restores."""
    import ctypes
    pm = _pm()
    with pm.Muca([prob]) as a:
        a.iterate(100)
        good = a.checkpoint()
        blob = bytearray(good)
        off = 32 + ctypes.sizeof(pm.Problem)          # header, then the problem, then the spins
        assert max(blob[off:off + prob.L * prob.L * prob.n_chains]) < prob.q
        blob[off + 5 * prob.n_chains + 3] = bad       # site 5 of chain 3
        with pm.Muca([prob]) as b:
            before = b.spins().copy()
            with pytest.raises(pm.MucaError, match="out of range"):
                b.restore(bytes(blob))
            assert np.array_equal(b.spins(), before)
            b.restore(good)
            assert np.array_equal(b.spins(), a.spins()) and np.array_equal(b.k(), a.k())


def test_restore_rejects_non_finite_weights():
    """A checkpoint whose log-weights hold a NaN or an infinity is refused on
    the host before any state changes."""
    import ctypes
    pm = _pm()
    prob = Problem(ISING, 8, 16, 73)
    with pm.Muca([prob]) as a:
        a.iterate(100)
        good = a.checkpoint()
        N, C = prob.L * prob.L, prob.n_chains
        off = 32 + ctypes.sizeof(pm.Problem) + N * C + 8 * C   # header, problem, spins, k and M
        for bad in (np.nan, np.inf, -np.inf):
            blob = bytearray(good)
            blob[off + 8 * 3:off + 8 * 4] = np.float64(bad).tobytes()   # lnW[3]
            with pm.Muca([prob]) as b:
                before, w_before = b.spins().copy(), b.lnW().copy()
                with pytest.raises(pm.MucaError, match="not finite"):
                    b.restore(bytes(blob))
                assert np.array_equal(b.spins(), before) and _same_bits(b.lnW(), w_before)
                b.restore(good)
                assert _same_bits(b.lnW(), a.lnW())


@pytest.mark.parametrize("prob,chunks", [(Problem(ISING, 64, 1, 74), 64), (Problem(ISING, 256, 1, 75), 1024)],
                         ids=["ising64", "ising256-generic"])
def test_launch_longer_than_the_chunk_counter_is_refused(prob, chunks):
    """The walkers count a launch's chunks in int32: a call whose sweeps would
    overflow that count is refused before any launch, and the sweep counter
    and the state stay as they were."""
    pm = _pm()
    with pm.Muca([prob]) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        cap = (2 ** 31 - 1) // chunks
        ctx.sweep(3, pm.REC_MUCA)
        before = (ctx.sweep_count(), ctx.spins().copy(), ctx.chain_hist().copy())
        for call in (lambda: ctx.sweep(cap + 1, pm.REC_MUCA), lambda: ctx.sweep(cap + 1, pm.REC_NONE),
                     lambda: ctx.iterate(cap + 1)):
            with pytest.raises(pm.MucaError, match="exceeds"):
                call()
        assert ctx.sweep_count() == before[0] == 3
        assert np.array_equal(ctx.spins(), before[1]) and np.array_equal(ctx.chain_hist(), before[2])
        with pytest.raises(pm.MucaError, match="out of range"):
            ctx.sweep(2 ** 30 + 1, pm.REC_NONE)
