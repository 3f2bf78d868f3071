"""GPU parity of the learned-initial-weights MLP against the float64
reference with matched bfloat16 rounding (through the C ABI): predictions,
gradients and an Adam step element by element (tolerances derived in
tests/mlp_check.py), the training trajectory against the reference's."""
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


@pytest.mark.parametrize("n,init", [(64, "normal"), (200, "normal"), (1000, "normal"), (6002, "normal"),
                                    (1000, "library"), (6002, "library")])
def test_forward_and_gradients_element_wise(n, init):
    """Every prediction and every gradient element against the reference at
    matched bfloat16 rounding, measured against its term scale (mlp_check):
    all within 2^-6 of the scale, at most half a per cent of a block beyond
    1e-3.  The same GPU results against a reference with a planted mistake
    (a shifted bias, two swapped rows of a 16 x 16 tile of W2) fail."""
    import mlp_check
    import paper_1212_3975_amd as pm
    x, t = _data(n, n + 1)
    with pm.Mlp(max_samples=8192, seed=n) as m:
        if init == "normal":
            rng = np.random.default_rng(n)
            m.set_params(rng.normal(0, 0.25, mlp_ref.N_PARAMS).astype(np.float32))
        p = m.params()
        y = m.predict(x)
        m.add_data(x, t)
        loss, g = m.gradients()
    p64, x64, t64 = p.astype(np.float64), x.astype(np.float64), t.astype(np.float64)
    yr, _ = mlp_ref.forward(p64, x64)
    lr_, gr = mlp_ref.loss_and_grad(p64, x64, t64)
    ys, gs = mlp_ref.term_scales(p64, x64, t64)
    ok, worst, n_out = mlp_check.compare(y, yr, ys)
    print(f"  y: worst {worst:.2e} of scale, {n_out} of {n} beyond 1e-3", flush=True)
    assert ok, (worst, n_out)
    ok, res = mlp_check.compare_grad(g, gr, gs)
    print("  grad:", {k: (f"{v[1]:.1e}", v[2]) for k, v in res.items()}, flush=True)
    assert ok, res
    assert loss == pytest.approx(lr_, rel=1e-3)
    d = mlp_ref.unpack(p64)
    shifted = dict(d, b2=np.roll(d["b2"], -1))
    swapped = dict(d, W2=d["W2"].copy())
    swapped["W2"][[3, 4]] = swapped["W2"][[4, 3]]
    for bad in (mlp_ref.pack(shifted), mlp_ref.pack(swapped)):
        yb, _ = mlp_ref.forward(bad, x64)
        _, gb = mlp_ref.loss_and_grad(bad, x64, t64)
        assert not mlp_check.compare(y, yb, ys)[0]
        assert not mlp_check.compare_grad(g, gb, gs)[0]


def test_adam_step_element_wise():
    """One Adam step from freshly set parameters: the bias-corrected first
    step moves each parameter by lr times the sign of its gradient, so every
    parameter whose gradient is clearly away from zero (beyond 2^-6 of its
    term scale, where the gradient check fixes the sign) lands where the
    reference's step puts it, to float32 rounding."""
    import paper_1212_3975_amd as pm
    x, t = _data(1000, 21)
    lr = 1e-3
    with pm.Mlp(max_samples=2048, seed=5) as m:
        p0 = m.params()
        m.add_data(x, t)
        m.train(1, lr)
        p1 = m.params()
    p64, x64, t64 = p0.astype(np.float64), x.astype(np.float64), t.astype(np.float64)
    _, gr = mlp_ref.loss_and_grad(p64, x64, t64)
    _, gs = mlp_ref.term_scales(p64, x64, t64)
    pr, _, _ = mlp_ref.adam(p64, gr, np.zeros_like(gr), np.zeros_like(gr), 1, lr)
    sure = np.abs(gr) > 2.0 ** -6 * gs
    assert sure.mean() > 0.8, sure.mean()
    err = np.abs(p1.astype(np.float64) - pr)[sure]
    assert np.all(err <= 4e-7 * (np.abs(p64[sure]) + lr)), err.max()
    # the rest (gradients near zero, whose sign rounding may decide) moved by
    # at most lr
    assert np.all(np.abs(p1.astype(np.float64) - p64)[~sure] <= lr * (1 + 1e-6) + 4e-7 * np.abs(p64[~sure]))


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
