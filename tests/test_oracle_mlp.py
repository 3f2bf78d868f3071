"""Pins of the reference MLP: its float64 gradient equals central finite
differences of its loss; bfloat16 rounding is round-to-nearest-even; its GELU
is within the tanh form's known error of the exact x*Phi(x); its Adam step
(Kingma and Ba) has the closed forms that bias correction gives."""
import numpy as np
from scipy.special import erf

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


def test_gelu_is_the_tanh_form_of_x_phi_x():
    """Hendrycks and Gimpel's tanh approximation stays within 5e-4 of the exact
    GELU x*Phi(x) (its largest error is 4.7e-4, near |x| = 2); a dropped cubic
    term errs by 3e-2 and a coefficient of 0.04 instead of 0.044715 by 3e-3.
    The derivative is within 1e-3 of the exact one, Phi(x) + x*phi(x)."""
    z = np.linspace(-8.0, 8.0, 20001)
    exact = 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))
    dexact = 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)
    val, der = mlp_ref.gelu(z)
    assert np.abs(val - exact).max() < 5e-4
    assert np.abs(der - dexact).max() < 1e-3
    v0, d0 = mlp_ref.gelu(np.array([0.0]))
    assert v0[0] == 0.0 and d0[0] == 0.5


def test_adam_first_step_moves_each_parameter_by_lr():
    """With bias correction the first step is lr * g / (|g| + eps): every
    parameter moves by lr against its gradient's sign, whatever its size
    (|g| >= 1e-3 here, so eps changes the step by at most 1e-5)."""
    rng = np.random.default_rng(5)
    p = rng.normal(0, 1, 1000)
    g = rng.choice([-1.0, 1.0], 1000) * 10.0 ** rng.uniform(-3, 3, 1000)
    lr = 1e-3
    p1, m, v = mlp_ref.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    np.testing.assert_allclose(p1 - p, -lr * np.sign(g), rtol=1e-4)
    p0, _, _ = mlp_ref.adam(p, np.zeros_like(p), np.zeros_like(p), np.zeros_like(p), 1, lr)
    assert np.array_equal(p0, p)


def test_adam_constant_gradient_gives_equal_steps():
    """Under a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step is lr * g / (|g| + eps); without the correction
    the first step would be (1 - b1) / sqrt(1 - b2) = 3.2 times that.  The
    step is unchanged when the gradient is scaled."""
    rng = np.random.default_rng(6)
    g = rng.choice([-1.0, 1.0], 64) * rng.uniform(0.1, 2.0, 64)
    lr = 3e-3
    for scale in (1.0, 1e3):
        p = np.zeros(64)
        m = np.zeros(64)
        v = np.zeros(64)
        for step in range(1, 60):
            p_new, m, v = mlp_ref.adam(p, scale * g, m, v, step, lr)
            np.testing.assert_allclose(p_new - p, -lr * np.sign(g), rtol=1e-6, atol=1e-12)
            p = p_new


def test_adam_impulse_response_decays_at_the_moment_rates():
    """A single gradient g at step 1 and zero gradients after it: the moments
    are then m_t = (1 - b1) b1^(t-1) g and v_t = (1 - b2) b2^(t-1) g^2, so the
    step at t is lr * sign(g) * c1_t / sqrt(c2_t) with c_t = b^(t-1) (1 - b) /
    (1 - b^t) for each rate (eps is negligible at |g| ~ 1).  This fixes which
    rate belongs to which moment, which a constant gradient does not."""
    b1, b2, lr = 0.9, 0.999, 1e-2
    g = np.array([1.3, -0.7])
    p = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 31):
        p_new, m, v = mlp_ref.adam(p, g if t == 1 else np.zeros(2), m, v, t, lr)
        c1 = b1 ** (t - 1) * (1 - b1) / (1 - b1 ** t)
        c2 = b2 ** (t - 1) * (1 - b2) / (1 - b2 ** t)
        np.testing.assert_allclose(p_new - p, -lr * np.sign(g) * c1 / np.sqrt(c2), rtol=1e-6)
        p = p_new


def test_term_scales_bound_the_values_and_equal_them_for_non_negative_terms():
    """The term scale of every output and gradient element is at least the
    element's magnitude (triangle inequality), and equals it when every term
    is non-negative: positive weights, inputs and biases keep every
    pre-activation and GELU derivative positive, and targets below the
    predictions make every back-propagated factor positive."""
    from oracle import mlp_ref
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (96, 4))
    t = rng.normal(0, 0.5, 96)
    p = rng.normal(0, 0.3, mlp_ref.N_PARAMS)
    ys, gs = mlp_ref.term_scales(p, x, t)
    y, _ = mlp_ref.forward(p, x)
    _, g = mlp_ref.loss_and_grad(p, x, t)
    assert np.all(ys >= np.abs(y) * (1 - 1e-12)) and np.all(gs >= np.abs(g) * (1 - 1e-12))
    assert np.any(gs > 2 * np.abs(g))   # mixed signs: the bound is not tight
    p = np.abs(p) + 0.01
    x = np.abs(x) + 0.01
    y, _ = mlp_ref.forward(p, x)
    t = y - 1.0
    ys, gs = mlp_ref.term_scales(p, x, t)
    _, g = mlp_ref.loss_and_grad(p, x, t)
    assert np.allclose(ys, np.abs(y), rtol=1e-12) and np.allclose(gs, np.abs(g), rtol=1e-12)


def test_elementwise_check_accepts_rounding_and_rejects_planted_mistakes():
    """The element-wise check used against the GPU: the reference at float32
    input precision passes against itself; a reference with a planted
    mistake (the bias of hidden unit o taken from o+1, two rows of the first
    16 x 16 tile of W2 swapped, or one sample's input misread) fails."""
    import mlp_check
    from oracle import mlp_ref
    rng = np.random.default_rng(9)
    n = 300
    x = np.stack([rng.integers(0, 2, n), rng.integers(0, 2, n), 8.0 / rng.choice([8, 16, 32], n),
                  rng.uniform(-2, 2, n)], axis=1)
    t = 0.3 * np.cos(x[:, 3])
    p = rng.normal(0, 0.25, mlp_ref.N_PARAMS).astype(np.float32).astype(np.float64)
    y, _ = mlp_ref.forward(p, x)
    _, g = mlp_ref.loss_and_grad(p, x, t)
    ys, gs = mlp_ref.term_scales(p, x, t)
    assert mlp_check.compare(y, y, ys)[0] and mlp_check.compare_grad(g, g, gs)[0]
    d = mlp_ref.unpack(p)
    shifted = dict(d, b2=np.roll(d["b2"], -1))
    swapped = dict(d, W2=d["W2"].copy())
    swapped["W2"][[3, 4]] = swapped["W2"][[4, 3]]
    for bad in (mlp_ref.pack(shifted), mlp_ref.pack(swapped)):
        yb, _ = mlp_ref.forward(bad, x)
        _, gb = mlp_ref.loss_and_grad(bad, x, t)
        assert not mlp_check.compare(yb, y, ys)[0]
        assert not mlp_check.compare_grad(gb, g, gs)[0]
    xb = x.copy()
    xb[17, 3] += 0.25
    yb, _ = mlp_ref.forward(p, xb)
    assert not mlp_check.compare(yb, y, ys)[0]
