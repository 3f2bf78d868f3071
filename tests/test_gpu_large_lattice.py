"""Parity of the walkers on the compact acceptance table (Ising L = 96 and
128, whose 32-bit tables do not fit in LDS beside the lattices, and 8-Potts
L = 48) against the oracle, through the C ABI.  Up to 32 chains per workgroup
the streamed walkers run these problems, above that the packed Ising and
byte-wise Potts walkers; the cases cover both.  The compact walkers decide
most moves from a 14-bit prefix of the threshold and redo a dword exactly
(full threshold from HBM, draw regenerated) when a draw's prefix equals it,
about once per 2^14 sites: at these sizes and lengths every test passes that
path hundreds of times, and every trajectory must still equal the oracle's bit
for bit."""
import ctypes

import numpy as np
import pytest

import oracle
from conftest import device_table, gpu_available
from workloads import ISING, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.uint64), np.asarray(b, np.float64).view(np.uint64))


def _compare(ctx, orc):
    assert np.array_equal(ctx.spins(), orc.spins), "spins differ"
    assert np.array_equal(ctx.k(), orc.k) and np.array_equal(ctx.m(), orc.m), "k or M differ"


PLACED = dict(rng_mode=4, spin_placement=1, table_placement=1)


@pytest.mark.parametrize("L,chains,cw", [(96, 40, 32), (96, 70, 64), (128, 40, 32), (128, 20, 16)],
                         ids=["L96-c40-cw32", "L96-c70-cw64", "L128-c40-cw32", "L128-c20-cw16"])
def test_compact_walker_iterations_bit_exact(L, chains, cw):
    """Weight iterations with the correction function (real weights from the
    second iteration on): per-chain and merged histograms, weights, tables,
    spins, k and M after each."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, chains, 90 + L + chains)
    with pm.Muca([prob], correction=1, chains_per_wg=cw, **PLACED) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["fast_walker"] == 1 and info["chains_per_wg"] == cw
        orc = oracle.OracleRun(prob.model, L, chains, prob.seed)
        for it in range(4):
            ctx.sweep(120, pm.REC_MUCA)
            ch = ctx.chain_hist()
            st = ctx.merge_update(True)[0]
            H, fl, per_chain = orc.iterate(120, correct=True)
            print(f"  iteration {it}: visited {fl.visited}", flush=True)
            assert np.array_equal(ch, per_chain), f"per-chain histograms differ at iteration {it}"
            assert np.array_equal(ctx.H(), H) and st["visited"] == fl.visited
            assert _same_bits(ctx.lnW(), orc.lnW)
            assert np.array_equal(ctx.table(), device_table(orc))
            _compare(ctx, orc)


@pytest.mark.parametrize("L", [96, 128])
def test_compact_walker_production_bit_exact(L):
    """Production under canonical weights near the critical point: counts and
    |M| sums per bin, bit for bit."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, 36, 7 + L)
    lnW = -0.43 * oracle.energies(ISING, L)
    with pm.Muca([prob], chains_per_wg=32, **PLACED) as ctx:
        assert ctx.launch_info()["fast_walker"] == 1
        ctx.set_log_weights(0, lnW)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed)
        orc.set_log_weights(lnW)
        ctx.clear_production()
        ctx.sweep(60, pm.REC_NONE)
        ctx.sweep(150, pm.REC_PROD)
        cnt, sab = orc.production(60, 150)
        assert np.array_equal(ctx.prod_counts(), cnt) and np.array_equal(ctx.prod_absm(), sab)
        _compare(ctx, orc)


def _checkpoint_with_spins(ctx, prob, spins_cn):
    """The context's checkpoint with its spins replaced ([C][N] -> the blob's
    [N][C] layout); k and M are recomputed on restore."""
    import paper_1212_3975_amd as pm
    blob = bytearray(ctx.checkpoint())
    off = 32 + ctypes.sizeof(pm.Problem)
    N, C = prob.L * prob.L, prob.n_chains
    blob[off:off + N * C] = np.ascontiguousarray(spins_cn.T).tobytes()
    return bytes(blob)


@pytest.mark.parametrize("L", [96, 128])
def test_compact_walker_at_both_ends_of_the_energy_range(L):
    """Chains started in the two ground states (k = 0, all spins equal) and in
    the two checkerboards (k = 2N), under weights that favour both ends,
    lnW(k) = 1.2 |k - N| (canonical at beta = 0.6 on either side, the ordered
    phase): moves from and next to the first and last table rows."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, L, 24, 300 + L)
    N = L * L
    k = np.arange(2 * N + 1)
    lnW = 1.2 * np.abs(k - N).astype(np.float64)
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    board = ((x + y) % 2).astype(np.uint8).ravel()
    spins = np.zeros((prob.n_chains, N), np.uint8)
    spins[6:12] = 1
    spins[12:18] = board
    spins[18:24] = 1 - board
    with pm.Muca([prob], chains_per_wg=32, **PLACED) as ctx:
        assert ctx.launch_info()["fast_walker"] == 1
        ctx.restore(_checkpoint_with_spins(ctx, prob, spins))
        ctx.set_log_weights(0, lnW)
        kk = ctx.k()
        assert np.all(kk[:12] == 0) and np.all(kk[12:] == 2 * N)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed)
        orc.spins[:] = spins
        for c in range(prob.n_chains):
            orc.k[c], orc.m[c] = oracle.energy(ISING, L, orc.spins[c])
        orc.set_log_weights(lnW)
        for rep in range(3):
            ctx.sweep(40, pm.REC_MUCA)
            orc.sweeps(40, oracle.REC_MUCA)
            assert np.array_equal(ctx.chain_hist(), orc.hist)
            _compare(ctx, orc)
        kk = ctx.k()
        print(f"  k after 120 sweeps: {kk.min()}..{kk.max()} of 0..{2 * N}", flush=True)
        assert kk[:12].max() < N // 2 and kk[12:].min() > 3 * N // 2


# ---------------------------------------------------------------- 8-state Potts L = 48

@pytest.mark.parametrize("chains,cw", [(40, 32), (20, 16), (35, 35)], ids=["c40-cw32", "c20-cw16", "c35-cw35"])
def test_compact_potts_walker_iterations_bit_exact(chains, cw):
    """8-state Potts L = 48 with the compact table: weight iterations with the
    correction function, every per-chain and merged histogram, weight, table
    and state bit for bit."""
    from workloads import POTTS
    import paper_1212_3975_amd as pm
    prob = Problem(POTTS, 48, chains, 500 + chains, q=8)
    with pm.Muca([prob], correction=1, chains_per_wg=cw, **PLACED) as ctx:
        info = ctx.launch_info()
        print("launch", info, flush=True)
        assert info["fast_walker"] == 1 and info["chains_per_wg"] == cw
        orc = oracle.OracleRun(prob.model, 48, chains, prob.seed, q=8)
        for it in range(4):
            ctx.sweep(150, pm.REC_MUCA)
            ch = ctx.chain_hist()
            st = ctx.merge_update(True)[0]
            H, fl, per_chain = orc.iterate(150, correct=True)
            print(f"  iteration {it}: visited {fl.visited}", flush=True)
            assert np.array_equal(ch, per_chain), f"per-chain histograms differ at iteration {it}"
            assert np.array_equal(ctx.H(), H) and st["visited"] == fl.visited
            assert _same_bits(ctx.lnW(), orc.lnW)
            assert np.array_equal(ctx.table(), device_table(orc))
            _compare(ctx, orc)


def test_compact_potts_walker_production_and_both_ends():
    """Production counts bit for bit, from chains started in ground states
    (k = 0, one colour) and two-colour checkerboards (k = 2N), under weights
    that favour both ends, lnW(k) = 1.5 |k - N| (canonical at beta = 1.5 on
    either side, beyond the transition at 1.3425)."""
    from workloads import POTTS
    import paper_1212_3975_amd as pm
    L = 48
    prob = Problem(POTTS, L, 24, 777, q=8)
    N = L * L
    k = np.arange(2 * N + 1)
    lnW = 1.5 * np.abs(k - N).astype(np.float64)
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    board = ((x + y) % 2).astype(np.uint8).ravel()
    spins = np.zeros((prob.n_chains, N), np.uint8)
    for c in range(12):
        spins[c] = c % 8                                # ground states of several colours
    for c in range(12, 24):
        spins[c] = np.where(board == 1, c % 8, (c + 3) % 8)   # two-colour checkerboards
    with pm.Muca([prob], chains_per_wg=32, **PLACED) as ctx:
        assert ctx.launch_info()["fast_walker"] == 1
        ctx.restore(_checkpoint_with_spins(ctx, prob, spins))
        ctx.set_log_weights(0, lnW)
        kk = ctx.k()
        assert np.all(kk[:12] == 0) and np.all(kk[12:] == 2 * N)
        orc = oracle.OracleRun(prob.model, L, prob.n_chains, prob.seed, q=8)
        orc.spins[:] = spins
        for c in range(prob.n_chains):
            orc.k[c], orc.m[c] = oracle.energy(POTTS, L, orc.spins[c])
        orc.set_log_weights(lnW)
        ctx.clear_production()
        ctx.sweep(30, pm.REC_NONE)
        ctx.sweep(120, pm.REC_PROD)
        cnt, _ = orc.production(30, 120)
        assert np.array_equal(ctx.prod_counts(), cnt)
        _compare(ctx, orc)
        kk = ctx.k()
        print(f"  k after 150 sweeps: {kk.min()}..{kk.max()} of 0..{2 * N}", flush=True)
        assert kk[:12].max() < N // 2 and kk[12:].min() > 3 * N // 2
