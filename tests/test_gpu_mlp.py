"""GPU parity of the learned-initial-weights MLP against the float64
reference with matched bfloat16 rounding (through the C ABI)."""
import numpy as np
import pytest

from conftest import gpu_available
from oracle import mlp_ref
from workloads import ISING, Problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _data(n, seed):
    rng = np.random.default_rng(seed)
    model = rng.integers(0, 2, n)
    L = rng.choice([8, 16, 24, 32, 48], n)
    e = rng.uniform(-2, 2, n)
    x = np.stack([(model == 0) * 1.0, (model == 1) * 1.0, 8.0 / L, e], axis=1)
    t = 0.35 * np.cos(e) + 0.1 * x[:, 2] + 0.05 * model
    return x.astype(np.float32), t.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [64, 200, 1000])
def test_forward_and_gradients_match_reference(n):
    import paper_1212_3975_amd as pm
    rng = np.random.default_rng(n)
    p = (rng.normal(0, 0.25, mlp_ref.N_PARAMS)).astype(np.float32)
    x, t = _data(n, n + 1)
    with pm.Mlp(max_samples=2048) as m:
        m.set_params(p)
        assert np.array_equal(m.params(), p)
        y = m.predict(x)
        yr, _ = mlp_ref.forward(p.astype(np.float64), x.astype(np.float64))
        assert np.max(np.abs(y - yr)) <= 2e-2 * max(1.0, np.max(np.abs(yr))), np.max(np.abs(y - yr))
        m.add_data(x, t)
        loss, g = m.gradients()
        lr_, gr = mlp_ref.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
        assert loss == pytest.approx(lr_, rel=2e-2)
        # every parameter block agrees to 2% in norm (bf16 rounding may fall
        # differently when float32 and float64 straddle a rounding boundary)
        for a, b in ((0, 256), (256, 320), (320, 4416), (4416, 4480), (4480, 8576), (8576, 8640), (8640, 8704),
                     (8704, 8705)):
            assert _rel(g[a:b], gr[a:b]) < 2e-2, (a, b, _rel(g[a:b], gr[a:b]))


def test_training_reduces_loss_like_reference_adam():
    import paper_1212_3975_amd as pm
    x, t = _data(700, 5)
    with pm.Mlp(max_samples=1024, seed=3) as m:
        p0 = m.params().astype(np.float64)
        m.add_data(x, t)
        losses = m.train(300, 3e-3)
        assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])
        # the reference network trained with the same Adam steps reaches a similar loss
        p, mm, vv = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        ref = []
        for step in range(1, 301):
            l, g = mlp_ref.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
            ref.append(l)
            p, mm, vv = mlp_ref.adam(p, g, mm, vv, step, 3e-3)
        assert losses[0] == pytest.approx(ref[0], rel=2e-2)
        assert losses[-1] < 3 * ref[-1] + 1e-4 and ref[-1] < 3 * losses[-1] + 1e-4


def test_learned_weights_round_trip_through_a_run():
    """Converged weights of a small run become training data (ln Omega / N,
    normalised to sum Omega = 2^N); the trained network's prediction, installed
    as lnW = -N f, follows the converged weights up to a constant."""
    import paper_1212_3975_amd as pm
    prob = Problem(ISING, 8, 64, 3)
    with pm.Muca([prob]) as ctx, pm.Mlp(max_samples=4096, seed=7) as m:
        for _ in range(25):
            st = ctx.iterate(2000)[0]
        assert st["flat"]
        lnW = ctx.lnW()
        mask = ctx.reachable()
        m.add_weights(ctx, 0)
        assert m.num_samples() == int(mask.sum())
        m.train(3000, 2e-3)
        m.set_log_weights(ctx, 0)
        pred = ctx.lnW()
        assert np.all(pred[~mask] == 0.0)
        d = (pred - lnW)[mask]
        d -= d.mean()
        assert np.max(np.abs(d)) < 2.0, np.max(np.abs(d))
        # the installed weights give a flat histogram within a few iterations
        flat_iters = next(i for i in range(1, 11) if ctx.iterate(2000)[0]["flat"])
        assert flat_iters <= 5
