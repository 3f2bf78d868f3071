"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark uses (tuned).  The oracle recomputes a sample of
chains one by one (a chain's trajectory depends only on the seed, its index
and lnW); everything else is checked through properties that hold at any
size: tracked energies equal a recompute from the spins, the merged histogram
sums to chains x sweeps and is empty on unreachable bins."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from workloads import C2, C3

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _recompute_k(spins_cn: np.ndarray, L: int) -> np.ndarray:
    s = spins_cn.reshape(-1, L, L)
    return ((s != np.roll(s, 1, axis=2)).sum(axis=(1, 2)) + (s != np.roll(s, 1, axis=1)).sum(axis=(1, 2))).astype(np.int32)


@pytest.mark.parametrize("plan", [C2, C3], ids=["ising64x4096", "potts32x4096"])
def test_first_iteration_sampled_chains(plan):
    import paper_1212_3975_amd as pm
    prob = plan.problems[0]
    M = plan.sweeps_per_iter
    with pm.Muca([prob]) as ctx:
        print("launch", ctx.launch_info(), flush=True)
        ctx.sweep(M, pm.REC_MUCA)
        ch = ctx.chain_hist()
        spins = ctx.spins()
        k = ctx.k()
        for c0, n in ((0, 32), (prob.n_chains - 32, 32)):
            print(f"  oracle chains {c0}..{c0 + n - 1}", flush=True)
            orc = oracle.OracleRun(prob.model, prob.L, n, prob.seed, q=prob.q, chain0=c0)
            orc.sweeps(M, oracle.REC_MUCA)
            assert np.array_equal(ch[c0:c0 + n], orc.hist)
            assert np.array_equal(spins[c0:c0 + n], orc.spins)
            assert np.array_equal(k[c0:c0 + n], orc.k)
        assert np.array_equal(_recompute_k(spins, prob.L), k)
        st = ctx.merge_update(True)[0]
        H = ctx.H()
        assert H.sum() == prob.n_chains * M == st["total"]
        assert np.all(H[~ctx.reachable()] == 0)
        assert np.array_equal(H, ch.astype(np.int64).sum(axis=0))
        # the weights follow the recursion from lnW = 0 on the merged histogram
        lnW = ctx.lnW()
        assert np.all(lnW[H == 0] == 0.0) and np.all(lnW[H > 0] <= 0.0)
        # a second iteration under the new weights keeps every invariant
        st2 = ctx.iterate(M)[0]
        assert st2["total"] == prob.n_chains * M
        assert np.array_equal(_recompute_k(ctx.spins(), prob.L), ctx.k())
        assert np.all(ctx.H()[~ctx.reachable()] == 0)


def test_mixed_batch_one_launch_sampled_chains():
    """The nine-problem batch in one tuned launch (Ising L = 16..64 and
    8-Potts L = 8..32, 512 chains each): per problem, eight chains recomputed
    by the oracle match bit for bit after one iteration of 2000 sweeps, and
    every chain keeps its invariants."""
    import paper_1212_3975_amd as pm
    from workloads import C4
    probs = list(C4.problems)
    M = C4.sweeps_per_iter
    with pm.Muca(probs, use_graph=1) as ctx:
        infos = [ctx.launch_info(i) for i in range(len(probs))]
        print("launch", infos, flush=True)
        ctx.sweep(M, pm.REC_MUCA)
        for j, prob in enumerate(probs):
            print(f"  problem {j}: model {prob.model} L {prob.L}", flush=True)
            ch = ctx.chain_hist(j)
            spins = ctx.spins(j)
            k = ctx.k(j)
            for c0 in (0, prob.n_chains - 4):
                orc = oracle.OracleRun(prob.model, prob.L, 4, prob.seed, q=prob.q, chain0=c0)
                orc.sweeps(M, oracle.REC_MUCA)
                assert np.array_equal(ch[c0:c0 + 4], orc.hist)
                assert np.array_equal(spins[c0:c0 + 4], orc.spins)
                assert np.array_equal(k[c0:c0 + 4], orc.k)
            assert np.array_equal(_recompute_k(spins, prob.L), k)
        st = ctx.merge_update(True)
        for j, prob in enumerate(probs):
            assert st[j]["total"] == prob.n_chains * M
        # the graph path continues from here with the same invariants
        st = ctx.iterate(M)
        for j, prob in enumerate(probs):
            assert st[j]["total"] == prob.n_chains * M
            assert np.array_equal(_recompute_k(ctx.spins(j), prob.L), ctx.k(j))
