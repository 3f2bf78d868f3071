"""Parity of the streamed Ising walker (Ising L = 64 with up to 16 chains per
workgroup, the benchmark's launch) against the oracle, through the C ABI.

Its helper waves form every dword's complete bulk from the row above as the
walker leaves it, and the two sides hand records and progress over through LDS
counters instead of barriers.  The cases cover one to four helper waves,
workgroups that are partly empty, chains split over several work items,
launches of a single sweep (the hand-over at launch start and end), production
(|M| with the last dword's flips still pending), and chains at both ends of the
energy range.  Every trajectory equals the oracle's bit for bit.  A last case
forces the bounded waits to give up at once and checks that the library
reports it instead of returning invalid chains."""
import ctypes

import numpy as np
import pytest

import oracle
from conftest import device_table, gpu_available
from workloads import ISING, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

STREAMED = 6   # muca_launch_info.walker of the streamed Ising walker


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64), np.asarray(b, np.float64).view(np.uint64))


def _compare_state(ctx, orc):
    assert np.array_equal(ctx.spins(), orc.spins), "spins differ"
    assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m), "k or M differ"


@pytest.mark.parametrize("chains,cw,rng_mode", [(1, 16, 2), (7, 16, 3), (16, 16, 4), (20, 16, 4), (37, 12, 2),
                                                (16, 16, 2), (16, 16, 5), (23, 12, 5)],
                         ids=["c1-one-helper", "c7-two-helpers", "c16-three-helpers", "c20-two-items",
                              "c37-cw12-one-helper", "c16-one-helper", "c16-four-helpers", "c23-cw12-four-helpers"])
def test_streamed_walker_iterations_bit_exact(chains, cw, rng_mode):
    """Two weight iterations with the correction function (real weights from
    the second on), then one launch of 400 sweeps: per-chain and merged
    histograms, weights, tables, spins, k and M after each."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 64, chains, 600 + chains + rng_mode)
    print("case", chains, cw, rng_mode, flush=True)
    with pm.Muca([prob], correction=1, chains_per_wg=cw, rng_mode=rng_mode, spin_placement=1,
                 table_placement=1) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["walker"] == STREAMED and info["rng_mode"] == rng_mode
        orc = oracle.OracleRun(prob.model, prob.L, chains, prob.seed)
        for it in range(2):
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
        ctx.sweep(400, pm.REC_MUCA)
        orc.hist[:] = 0
        orc.sweeps(400, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


def test_streamed_walker_single_sweep_launches():
    """Thirty launches of one sweep each under canonical weights near the
    critical point (every launch starts and ends the hand-over), recorded."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 64, 16, 611)
    lnW = -0.44 * oracle.energies(ISING, 64)
    with pm.Muca([prob], chains_per_wg=16, rng_mode=4, spin_placement=1, table_placement=1) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, prob.L, prob.n_chains, prob.seed)
        orc.set_log_weights(lnW)
        for _ in range(30):
            ctx.sweep(1, pm.REC_MUCA)
            orc.sweeps(1, oracle.REC_MUCA)
        assert np.array_equal(ctx.chain_hist(), orc.hist)
        _compare_state(ctx, orc)


def test_streamed_walker_production_bit_exact():
    """Production under canonical weights: counts and |M| sums per bin (|M| is
    counted while the sweep's last dword still holds its flips back)."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 64, 16, 612)
    lnW = -0.43 * oracle.energies(ISING, 64)
    with pm.Muca([prob], chains_per_wg=16, rng_mode=3, spin_placement=1, table_placement=1) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, prob.L, prob.n_chains, prob.seed)
        orc.set_log_weights(lnW)
        ctx.clear_production()
        ctx.sweep(60, pm.REC_NONE)
        ctx.sweep(150, pm.REC_PROD)
        cnt, sab = orc.production(60, 150)
        assert np.array_equal(ctx.prod_counts(), cnt) and np.array_equal(ctx.prod_absm(), sab)
        _compare_state(ctx, orc)


def _checkpoint_with_spins(ctx, prob, spins_cn):
    """The context's checkpoint with its spins replaced ([C][N] -> the blob's
    [N][C] layout); k and M are recomputed on restore."""
    import paper_1212_3975_amd as pm
    blob = bytearray(ctx.checkpoint())
    off = 32 + ctypes.sizeof(pm.Problem)
    N, C = prob.L * prob.L, prob.n_chains
    blob[off:off + N * C] = np.ascontiguousarray(spins_cn.T).tobytes()
    return bytes(blob)


def test_streamed_walker_at_both_ends_of_the_energy_range():
    """Chains started in the two ground states (k = 0) and the two
    checkerboards (k = 2N) under lnW(k) = 1.2 |k - N|, which keeps them near
    their ends: moves from and next to the first and last table rows."""
    import paper_1212_3975_amd as pm
    L = 64
    prob = Problem(ISING, L, 16, 613)
    N = L * L
    lnW = 1.2 * np.abs(np.arange(2 * N + 1) - N).astype(np.float64)
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    board = ((x + y) % 2).astype(np.uint8).ravel()
    spins = np.zeros((16, N), np.uint8)
    spins[4:8] = 1
    spins[8:12] = board
    spins[12:16] = 1 - board
    with pm.Muca([prob], chains_per_wg=16, rng_mode=4, spin_placement=1, table_placement=1) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED
        ctx.restore(_checkpoint_with_spins(ctx, prob, spins))
        ctx.set_log_weights(0, lnW)
        kk = ctx.k()
        assert np.all(kk[:8] == 0) and np.all(kk[8:] == 2 * N)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed)
        orc.spins[:] = spins
        for c in range(prob.n_chains):
            orc.k[c], orc.m[c] = oracle.energy(ISING, L, orc.spins[c])
        orc.set_log_weights(lnW)
        for _ in range(3):
            ctx.sweep(40, pm.REC_MUCA)
            orc.sweeps(40, oracle.REC_MUCA)
            assert np.array_equal(ctx.chain_hist(), orc.hist)
            _compare_state(ctx, orc)
        kk = ctx.k()
        print(f"  k after 120 sweeps: {kk.min()}..{kk.max()} of 0..{2 * N}", flush=True)
        assert kk[:8].max() < N // 2 and kk[8:].min() > 3 * N // 2


def test_expired_wait_is_reported():
    """With no polls allowed, the first wait of every workgroup gives up at
    once: the workgroups stop walking, the launch still ends, and the next call
    that reads results reports the expiry instead of returning the chains."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 64, 16, 614)
    with pm.Muca([prob], chains_per_wg=16, rng_mode=4, spin_placement=1, table_placement=1, wait_polls=-1) as ctx:
        assert ctx.launch_info()["walker"] == STREAMED
        ctx.sweep(5, pm.REC_MUCA)
        with pytest.raises(pm.MucaError, match="bounded wait"):
            ctx.merge_update(True)
        with pytest.raises(pm.MucaError, match="bounded wait"):
            ctx.spins()
    # the device is unharmed: a context with the default limit walks bit-exactly
    with pm.Muca([prob], chains_per_wg=16, rng_mode=4, spin_placement=1, table_placement=1) as ctx:
        ctx.sweep(20, pm.REC_MUCA)
        orc = oracle.OracleRun(prob.model, prob.L, prob.n_chains, prob.seed)
        orc.sweeps(20, oracle.REC_MUCA)
        _compare_state(ctx, orc)
