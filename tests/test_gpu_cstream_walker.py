"""Parity of the streamed Ising walkers on bit lattices against the oracle,
through the C ABI: on the compact table at L = 96 and 128 with up to 32
chains per workgroup (at L = 128 a ring of 16 record slots per lane, shorter
than a row), and on the 32-bit table at L = 64 with 17 to 64 chains per
workgroup.

Its helper waves form every dword's complete record from the bit lattices
(draw prefixes, then column codes, row steps and decode codes of both
candidates) once the walker has left the row above; the walker xors each
dword's flips into the bit lattice as a nibble.  The cases cover one to four
helper waves, partly empty workgroups, chains split over work items, launches
of a single sweep near the critical point (ties with the 14-bit entries are
redone exactly) and an expired bounded wait.  Production and chains at both
ends of the energy range run through this walker in the compact-table tests."""
import numpy as np
import pytest

import oracle
from conftest import device_table, gpu_available
from workloads import ISING, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

STREAMED_COMPACT_ISING = 8   # muca_launch_info.walker of the streamed compact Ising walker
STREAMED_BIT_ISING = 9       # the same walker on the 32-bit table (L = 64)
PLACED = dict(spin_placement=1, table_placement=1)


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64), np.asarray(b, np.float64).view(np.uint64))


def _compare_state(ctx, orc):
    assert np.array_equal(ctx.spins(), orc.spins), "spins differ"
    assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m), "k or M differ"


@pytest.mark.parametrize("L,chains,cw,rng_mode", [(96, 1, 32, 2), (96, 9, 16, 3), (96, 32, 32, 5), (96, 40, 32, 4),
                                                  (96, 23, 12, 2), (128, 1, 32, 2), (128, 32, 32, 5),
                                                  (128, 40, 32, 3), (64, 17, 32, 2), (64, 64, 64, 5),
                                                  (64, 70, 64, 4), (64, 48, 24, 3)],
                         ids=["L96-c1-one-helper", "L96-c9-two-helpers", "L96-c32-four-helpers", "L96-c40-two-items",
                              "L96-c23-cw12-one-helper", "L128-c1-one-helper", "L128-c32-four-helpers",
                              "L128-c40-two-items", "L64-c17-one-helper", "L64-c64-four-helpers",
                              "L64-c70-with-a-byte-walker-item", "L64-c48-cw24-two-helpers"])
def test_streamed_compact_ising_iterations_bit_exact(L, chains, cw, rng_mode):
    """Three weight iterations with the correction function (real weights from
    the second on), then one launch of 200 sweeps: per-chain and merged
    histograms, weights, tables, spins, k and M after each."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, chains, 800 + L + chains + rng_mode)
    print("case", L, chains, cw, rng_mode, flush=True)
    with pm.Muca([prob], correction=1, chains_per_wg=cw, rng_mode=rng_mode, **PLACED) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["walker"] == (STREAMED_BIT_ISING if L == 64 else STREAMED_COMPACT_ISING)
        assert info["rng_mode"] == rng_mode
        orc = oracle.OracleRun(prob.model, L, chains, prob.seed)
        for it in range(3):
            ctx.sweep(120, pm.REC_MUCA)
            ch = ctx.chain_hist()
            st = ctx.merge_update(True)[0]
            H, fl, per_chain = orc.iterate(120, correct=True)
            print(f"  iteration {it}: visited {fl.visited}", flush=True)
            assert np.array_equal(ch, per_chain), f"per-chain histograms differ at iteration {it}"
            assert np.array_equal(ctx.H(), H) and st["visited"] == fl.visited
            assert _same_bits(ctx.lnW(), orc.lnW)
            assert np.array_equal(ctx.table(), device_table(orc))
            _compare_state(ctx, orc)
        ctx.sweep(200, pm.REC_MUCA)
        orc.hist[:] = 0
        orc.sweeps(200, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


@pytest.mark.parametrize("L", [96, 128, 64])
def test_streamed_compact_ising_single_sweep_launches_near_the_critical_point(L):
    """Thirty launches of one sweep each under canonical weights at beta = 0.44
    (every launch starts and ends the hand-over; some draws tie with their
    14-bit entries and are redone)."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, 32, 811 + L)
    lnW = -0.44 * oracle.energies(ISING, L)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == (STREAMED_BIT_ISING if L == 64 else STREAMED_COMPACT_ISING)
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed)
        orc.set_log_weights(lnW)
        for _ in range(30):
            ctx.sweep(1, pm.REC_MUCA)
            orc.sweeps(1, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


@pytest.mark.parametrize("L", [64, 96])
def test_streamed_bit_ising_production_bit_exact(L):
    """Production under canonical weights near the critical point: counts and
    |M| sums per bin (|M| counted while the sweep's last dword still holds its
    flips back)."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, 48, 820 + L)
    lnW = -0.43 * oracle.energies(ISING, L)
    with pm.Muca([prob], chains_per_wg=48 if L == 64 else 32, rng_mode=4, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == (STREAMED_BIT_ISING if L == 64 else STREAMED_COMPACT_ISING)
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed)
        orc.set_log_weights(lnW)
        ctx.clear_production()
        ctx.sweep(50, pm.REC_NONE)
        ctx.sweep(120, pm.REC_PROD)
        cnt, sab = orc.production(50, 120)
        assert np.array_equal(ctx.prod_counts(), cnt) and np.array_equal(ctx.prod_absm(), sab)
        _compare_state(ctx, orc)


def test_streamed_compact_ising_expired_wait_is_reported():
    """With no polls allowed every workgroup's first wait gives up at once: the
    launch still ends, and the next call that reads results reports it."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 96, 32, 813)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, wait_polls=-1, **PLACED) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED_COMPACT_ISING
        ctx.sweep(3, pm.REC_MUCA)
        with pytest.raises(pm.MucaError, match="bounded wait"):
            ctx.merge_update(True)
    with pm.Muca([prob], chains_per_wg=32, rng_mode=5, **PLACED) as ctx:
        ctx.sweep(10, pm.REC_MUCA)
        orc = oracle.OracleRun(prob.model, 96, prob.n_chains, prob.seed)
        orc.sweeps(10, oracle.REC_MUCA)
        _compare_state(ctx, orc)
