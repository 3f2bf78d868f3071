"""Parity of the streamed compact 8-Potts walker (L = 48 with up to 32 chains
per workgroup) against the oracle, through the C ABI.

Its helper waves form every dword's complete record (draw prefixes, column
codes, row steps and decode codes of both candidates, and the state xor of the
proposals) once the walker has left the row above, drawing the previous
dword's last proposal again for the first site's left neighbour.  The cases
cover one to four helper waves, partly empty workgroups, chains split over
work items, launches of a single sweep, weights near the transition (where
draws that the compact entry cannot decide are redone exactly), production
counts and an expired bounded wait."""
import numpy as np
import pytest

import oracle
from conftest import device_table, gpu_available
from workloads import POTTS, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

STREAMED_POTTS = 7   # muca_launch_info.walker of the streamed compact Potts walker
PLACED = dict(spin_placement=1, table_placement=1)


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64), np.asarray(b, np.float64).view(np.uint64))


def _compare_state(ctx, orc):
    assert np.array_equal(ctx.spins(), orc.spins), "spins differ"
    assert np.array_equal(ctx.k(), orc.k), "k differs"


@pytest.mark.parametrize("chains,cw,rng_mode", [(1, 32, 2), (7, 16, 3), (32, 32, 5), (40, 32, 4), (23, 12, 2)],
                         ids=["c1-one-helper", "c7-two-helpers", "c32-four-helpers", "c40-two-items",
                              "c23-cw12-one-helper"])
def test_streamed_potts_iterations_bit_exact(chains, cw, rng_mode):
    """Three weight iterations with the correction function (real weights from
    the second on), then one launch of 300 sweeps: per-chain and merged
    histograms, weights, tables, spins and k after each."""
    import paper_1212_3975_amd as pm
    prob = Problem(POTTS, 48, chains, 700 + chains + rng_mode, q=8)
    print("case", chains, cw, rng_mode, flush=True)
    with pm.Muca([prob], correction=1, chains_per_wg=cw, rng_mode=rng_mode, **PLACED) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["walker"] == STREAMED_POTTS and info["rng_mode"] == rng_mode
        orc = oracle.OracleRun(prob.model, 48, chains, prob.seed, q=8)
        for it in range(3):
            ctx.sweep(150, pm.REC_MUCA)
            ch = ctx.chain_hist()
            st = ctx.merge_update(True)[0]
            H, fl, per_chain = orc.iterate(150, correct=True)
            print(f"  iteration {it}: visited {fl.visited}", flush=True)
            assert np.array_equal(ch, per_chain), f"per-chain histograms differ at iteration {it}"
            assert np.array_equal(ctx.H(), H) and st["visited"] == fl.visited
            assert _same_bits(ctx.lnW(), orc.lnW)
            assert np.array_equal(ctx.table(), device_table(orc))
            _compare_state(ctx, orc)
        ctx.sweep(300, pm.REC_MUCA)
        orc.hist[:] = 0
        orc.sweeps(300, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


def test_streamed_potts_single_sweep_launches_near_the_transition():
    """Forty launches of one sweep each under canonical weights at beta = 1.3
    (every launch starts and ends the hand-over; with thresholds away from 0
    and 2^32 - 1, some draws tie with their 14-bit entries and are redone)."""
    import paper_1212_3975_amd as pm
    prob = Problem(POTTS, 48, 32, 711, q=8)
    lnW = -1.3 * oracle.energies(POTTS, 48)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED_POTTS
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, 48, prob.n_chains, prob.seed, q=8)
        orc.set_log_weights(lnW)
        for _ in range(40):
            ctx.sweep(1, pm.REC_MUCA)
            orc.sweeps(1, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


def test_streamed_potts_production_counts():
    """Production under canonical weights at beta = 1.35: counts per bin."""
    import paper_1212_3975_amd as pm
    prob = Problem(POTTS, 48, 32, 712, q=8)
    lnW = -1.35 * oracle.energies(POTTS, 48)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=4, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED_POTTS
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, 48, prob.n_chains, prob.seed, q=8)
        orc.set_log_weights(lnW)
        ctx.clear_production()
        ctx.sweep(40, pm.REC_NONE)
        ctx.sweep(120, pm.REC_PROD)
        cnt, _ = orc.production(40, 120)
        assert np.array_equal(ctx.prod_counts(), cnt)
        _compare_state(ctx, orc)


def test_streamed_potts_expired_wait_is_reported():
    """With no polls allowed every workgroup's first wait gives up at once: the
    launch still ends, and the next call that reads results reports it."""
    import paper_1212_3975_amd as pm
    prob = Problem(POTTS, 48, 32, 713, q=8)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, wait_polls=-1, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED_POTTS
        ctx.sweep(3, pm.REC_MUCA)
        with pytest.raises(pm.MucaError, match="bounded wait"):
            ctx.merge_update(True)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, **PLACED) as ctx:
        ctx.sweep(10, pm.REC_MUCA)
        orc = oracle.OracleRun(prob.model, 48, prob.n_chains, prob.seed, q=8)
        orc.sweeps(10, oracle.REC_MUCA)
        _compare_state(ctx, orc)
