"""mucaReweightStatic, the entry point that allocates nothing, against
mucaReweight on the same production data (through the C ABI): bit for bit,
and within 1e-10 of the oracle's reweighting, over consecutive calls whose
inputs shrink (so stale contents of the static array would show)."""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from workloads import C2, ISING, POTTS, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _production(pm, prob, betas):
    """A short weight iteration with the correction function, then production;
    the context's own reweighting and the data it used."""
    with pm.Muca([prob], correction=1) as ctx:
        for _ in range(4):
            ctx.iterate(500)
        ctx.clear_production()
        ctx.sweep(100, pm.REC_NONE)
        ctx.sweep(400, pm.REC_PROD)
        res = ctx.reweight(0, betas)
        data = (ctx.lnW(), ctx.prod_counts(), ctx.prod_absm())
    return res, data


def _same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def test_static_reweighting_equals_context_reweighting_over_shrinking_calls():
    import paper_1212_3975_amd as pm
    cases = [(Problem(ISING, 16, 64, 81), np.array(C2.betas)),         # 513 bins, 200 beta
             (Problem(ISING, 8, 32, 82), np.linspace(0.2, 0.7, 7)),     # 129 bins, 7 beta
             (Problem(POTTS, 6, 48, 83, q=8), np.linspace(1.0, 1.6, 5))]  # 73 bins, 5 beta
    runs = [(prob, betas) + _production(pm, prob, betas) for prob, betas in cases]
    for rep in range(2):   # the largest call again after the smaller ones
        for prob, betas, (e, c, m), (lnW, cnt, sab) in runs:
            print(f"  call {rep}: model {prob.model} L {prob.L}, {cnt.size} bins, {betas.size} beta", flush=True)
            es, cs, ms = pm.reweight_static(prob.model, prob.L, lnW, cnt, sab if prob.model == ISING else None,
                                            betas)
            assert _same_bits(es, e) and _same_bits(cs, c)
            if prob.model == ISING:
                assert _same_bits(ms, m)
                eo, co, mo = oracle.reweight(prob.model, prob.L, lnW, cnt, sab, betas)
            else:
                assert np.all(np.isnan(ms)) and np.all(np.isnan(m))
                eo, co, mo = oracle.reweight(prob.model, prob.L, lnW, cnt, np.zeros_like(cnt), betas)
            for got, want in ((es, eo), (cs, co)) + (((ms, mo),) if prob.model == ISING else ()):
                assert np.all(np.abs(got - want) <= 1e-10 * np.abs(want)), float(np.max(np.abs(got - want)))
