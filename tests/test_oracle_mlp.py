"""Pins of the reference MLP: its float64 gradient equals central finite
differences of its loss; bfloat16 rounding is round-to-nearest-even."""
import numpy as np

from oracle import mlp_ref


def _data(n=37, seed=0):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(0, 2, n), rng.integers(0, 2, n), rng.uniform(0.06, 1, n),
                  rng.uniform(-2, 2, n)], axis=1).astype(np.float64)
    t = np.sin(x[:, 3]) * 0.3 + x[:, 2] * 0.1
    p = rng.normal(0, 0.3, mlp_ref.N_PARAMS)
    return p, x, t


def test_gradient_matches_finite_differences():
    p, x, t = _data()
    _, g = mlp_ref.loss_and_grad(p, x, t, round_bf16=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(256, 6), 256 + rng.choice(64, 3), 320 + rng.choice(4096, 8),
                          4416 + rng.choice(64, 3), 4480 + rng.choice(4096, 8), 8576 + rng.choice(64, 3),
                          8640 + rng.choice(64, 4), [8704]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp_ref.loss_and_grad(pp, x, t, False)[0] - mlp_ref.loss_and_grad(pm, x, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_bf16_rounding_is_nearest_even():
    """bfloat16 keeps 8 significant bits: the ulp at 1 is 2^-7.  Halfway
    cases go to the even neighbour, others to the nearest."""
    u = 2.0 ** -7
    cases = {1.0: 1.0, 1.0 + u / 2: 1.0, 1.0 + 3 * u / 2: 1.0 + 2 * u,
             1.0 + u / 2 + u / 8: 1.0 + u, -2.5: -2.5, 3.140625: 3.140625}
    for v, want in cases.items():
        assert mlp_ref.bf16(np.array([v]))[0] == want, v
    rng = np.random.default_rng(3)
    v = rng.normal(0, 10, 10000)
    assert np.all(np.abs(mlp_ref.bf16(v) - v) <= np.abs(v) * 2.0 ** -8)
