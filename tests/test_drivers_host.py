"""Host-side helpers of the drivers, no GPU: of the interface-tension driver
(Sec. 5) the 1/L fit, the per-site carry-over of converged weights between
lattice sizes and the 8-state Potts transition point; of the learned-weights
driver the loop that iterates to a flat histogram."""
import math

import numpy as np
import pytest

from paper_1212_3975_amd.interface_tension import BETA0, fit_inverse_l, rescaled_weights


def test_transition_point_is_the_self_dual_point():
    """The q-state Potts model with E = -sum of delta over bonds is self-dual
    where (e^beta - 1)^2 = q; for q = 8 that is ln(1 + sqrt 8)."""
    assert (math.exp(BETA0) - 1.0) ** 2 == pytest.approx(8.0, rel=1e-14)


def test_inverse_l_fit_recovers_exact_data():
    Ls = [16, 24, 32, 48, 64]
    s_inf, a = fit_inverse_l(Ls, [0.0372 + 0.81 / L for L in Ls])
    assert s_inf == pytest.approx(0.0372, abs=1e-13) and a == pytest.approx(0.81, rel=1e-12)
    # two points determine the line
    s_inf, a = fit_inverse_l([20, 40], [0.5, 0.3])
    assert s_inf == pytest.approx(0.1, abs=1e-13) and a == pytest.approx(8.0, rel=1e-12)


def test_inverse_l_fit_is_least_squares():
    """The residual of the fit is orthogonal to both basis functions."""
    rng = np.random.default_rng(4)
    Ls = np.array([16, 20, 24, 32, 40, 48])
    sig = 0.05 + 0.6 / Ls + rng.normal(0, 1e-3, Ls.size)
    s_inf, a = fit_inverse_l(Ls, sig)
    r = sig - (s_inf + a / Ls)
    assert abs(r.sum()) < 1e-12 and abs((r / Ls).sum()) < 1e-13


@pytest.mark.parametrize("L", [8, 16, 24])
def test_rescaled_weights_identity_at_the_same_size(L):
    rng = np.random.default_rng(L)
    lnW = rng.normal(0, 50, 2 * L * L + 1)
    np.testing.assert_allclose(rescaled_weights(lnW, L, L), lnW, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("Lp,L", [(16, 24), (24, 32), (32, 16)])
def test_rescaled_weights_keep_weights_linear_in_energy_per_site(Lp, L):
    """Weights c E + d N (a canonical weight plus a constant per site) carry
    over exactly: ln W / N as a function of E / N is the same line at every
    size.  Bins are k = 0..2N with E = -2N + k."""
    c, d = -1.31, 0.47
    Np, N = Lp * Lp, L * L
    E_prev = -2.0 * Np + np.arange(2 * Np + 1)
    E_new = -2.0 * N + np.arange(2 * N + 1)
    out = rescaled_weights(c * E_prev + d * Np, Lp, L)
    assert out.shape == (2 * N + 1,)
    np.testing.assert_allclose(out, c * E_new + d * N, rtol=1e-12, atol=1e-9)


def test_rescaled_weights_keep_the_per_site_values_at_shared_energies():
    """Where E / N of the new size falls on a bin of the old one (every
    fourth bin from L = 16 to L = 32, since N grows fourfold), the per-site
    value is that bin's; halfway between two of them it is their mean."""
    rng = np.random.default_rng(9)
    Lp, L = 16, 32
    Np, N = Lp * Lp, L * L
    lnW = np.cumsum(rng.normal(0, 3, 2 * Np + 1))
    out = rescaled_weights(lnW, Lp, L)
    np.testing.assert_allclose(out[::4] / N, lnW / Np, rtol=1e-12, atol=1e-12)
    mid = out[2::4][: 2 * Np] / N
    np.testing.assert_allclose(mid, 0.5 * (lnW[:-1] + lnW[1:]) / Np, rtol=1e-12, atol=1e-12)


class _ScriptedContext:
    """Stands in for a library context: iterate() returns scripted flatness."""

    def __init__(self, flats):
        self.flats = list(flats)
        self.calls = []

    def iterate(self, sweeps):
        self.calls.append(sweeps)
        flat = self.flats[len(self.calls) - 1]
        return [{"visited": 10, "reachable": 12, "min_over_max": 0.6 if flat else 0.1, "flat": flat}]


def test_iterate_to_flat_stops_at_the_first_flat_iteration():
    from paper_1212_3975_amd.learned_init import iterate_to_flat
    ctx = _ScriptedContext([False, False, True, True])
    n, hist = iterate_to_flat(ctx, 500, cap=10, label="t")
    assert n == 3 and len(hist) == 3 and ctx.calls == [500, 500, 500]
    assert [h["it"] for h in hist] == [1, 2, 3] and hist[-1]["flat"]


def test_iterate_to_flat_respects_the_cap_and_the_time_limit():
    from paper_1212_3975_amd.learned_init import iterate_to_flat
    ctx = _ScriptedContext([False] * 20)
    n, hist = iterate_to_flat(ctx, 100, cap=7, label="t")
    assert n is None and len(hist) == 7 and len(ctx.calls) == 7
    ctx = _ScriptedContext([False] * 20)
    n, hist = iterate_to_flat(ctx, 100, cap=7, label="t", max_seconds=-1.0)
    assert n is None and hist == [] and ctx.calls == []


def test_training_needs_three_steps():
    from paper_1212_3975_amd.learned_init import train
    with pytest.raises(ValueError, match="at least 3"):
        train("/nonexistent", chains=4, sweeps_ising=1, sweeps_potts=1, cap=1, refine=0, steps=2, max_seconds=1.0)
