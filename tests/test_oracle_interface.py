"""Pins of the oracle's interface-tension analysis (Sec. 5, Eq. 9).

The pin is a closed form.  Take a density of states ln Omega(E) = b* E + f(k)
with f(k) = h cos(2 pi (k - k1) / P) on a window of bins symmetric about
k1 + P/2, and give every bin the same count with lnW = -ln Omega (a flat
multicanonical histogram).  The reweighted log-probability at beta is then
f(k) + (b* - beta) E_k.  At beta = b*, it has two equal peaks of height h, at
k1 and k1 + P, and the minimum -h halfway between them.  So the equal-height
beta is b*, and sigma_od = (h - (-h)) / (2L) = h / L.  A wrong sign of
beta E, a dropped ln cnt, a wrong factor in 1/(2L) or an unequal-height beta
each move one of these values.

Wide brackets are pinned too: there the tilt (beta - b*) E makes one phase
dominate at most beta of the bracket, so a split between the peaks that moves
with beta (at the mean of the reweighted distribution) lands inside the
dominant peak and finds a false crossing.  The split at the valley, fixed in
k, does not.  Nor does a dip in a sparsely sampled tail or a lone ground-state
bin take the split: the two phases carry comparable probability, they do not.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import ISING, POTTS

B0_POTTS8 = math.log(1.0 + math.sqrt(8.0))   # Sec. 3: first-order transition of the 8-state Potts model


def double_well(model, L, k1, period, h, beta_star, counts=None):
    N = L * L
    nb = 2 * N + 1
    E = oracle.energies(model, L)
    k = np.arange(nb)
    lo, hi = k1 - period // 2 + 1, k1 + period + period // 2 - 1
    ln_omega = beta_star * E + h * np.cos(2.0 * np.pi * (k - k1) / period)
    cnt = np.zeros(nb, np.int64)
    cnt[lo:hi + 1] = 1 if counts is None else counts[lo:hi + 1]
    lnW = -ln_omega + np.log(np.maximum(cnt, 1))   # flat in the recorded counts' units
    return lnW, cnt


@pytest.mark.parametrize("model,L,k1,period", [(POTTS, 8, 30, 40), (POTTS, 12, 60, 80), (ISING, 8, 20, 30)])
@pytest.mark.parametrize("tilt", [0.0, 0.037, -0.11])
def test_equal_height_closed_form(model, L, k1, period, tilt):
    h = 1.7
    beta_star = B0_POTTS8 + tilt
    lnW, cnt = double_well(model, L, k1, period, h, beta_star)
    beta, sigma, ks = oracle.interface_tension(model, L, lnW, cnt, beta_star - 0.04, beta_star + 0.03)
    assert beta == pytest.approx(beta_star, abs=1e-12)
    assert sigma == pytest.approx(h / L, rel=1e-12)
    assert ks == (k1, k1 + period // 2, k1 + period)


def test_equal_height_uses_the_counts():
    # uneven counts with lnW carrying the same factor describe the same ensemble
    rng = np.random.default_rng(5)
    L, k1, period = 8, 30, 40
    counts = rng.integers(50, 5000, size=2 * L * L + 1)
    lnW, cnt = double_well(POTTS, L, k1, period, 1.3, B0_POTTS8, counts)
    beta, sigma, ks = oracle.interface_tension(POTTS, L, lnW, cnt, B0_POTTS8 - 0.04, B0_POTTS8 + 0.03)
    assert beta == pytest.approx(B0_POTTS8, abs=1e-12)
    assert sigma == pytest.approx(1.3 / L, rel=1e-12)
    # the same weights read with unit counts (ln cnt dropped, a plausible slip)
    # describe another ensemble and give another answer
    try:
        b2, s2, _ = oracle.interface_tension(POTTS, L, lnW, np.where(cnt > 0, 1, 0), B0_POTTS8 - 0.04,
                                             B0_POTTS8 + 0.03)
    except ValueError:   # no crossing in the bracket at all
        return
    assert abs(b2 - beta) > 1e-6 or abs(s2 - sigma) > 1e-6


def test_equal_height_with_a_long_disordered_tail():
    # Potts-like asymmetry: a long declining tail on the high-energy side puts
    # the middle of the sampled range beyond both peaks; the valley split
    # still falls between them
    L, k1, period, h, tail = 12, 60, 80, 1.9, 100
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    lo, hi = k1 - period // 2 + 1, k1 + period + period // 2 - 1
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k > hi, f[hi] - 0.05 * (k - hi), f)
    cnt = np.zeros(2 * N + 1, np.int64)
    cnt[lo:hi + tail + 1] = 1
    assert (lo + hi + tail) // 2 > k1 + period
    lnW = -(B0_POTTS8 * E + f)
    beta, sigma, ks = oracle.interface_tension(POTTS, L, lnW, cnt, B0_POTTS8 - 0.02, B0_POTTS8 + 0.015)
    assert beta == pytest.approx(B0_POTTS8, abs=1e-12)
    assert sigma == pytest.approx(h / L, rel=1e-12)
    assert ks == (k1, k1 + period // 2, k1 + period)


def test_equal_height_refuses_one_peak_and_a_bad_bracket():
    L = 8
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    ln_omega = B0_POTTS8 * E - 0.01 * (k - 60.0) ** 2   # one peak
    cnt = np.ones(2 * N + 1, np.int64)
    with pytest.raises(ValueError):
        oracle.interface_tension(POTTS, L, -ln_omega, cnt, B0_POTTS8 - 0.2, B0_POTTS8 + 0.2)
    # both ends above the equal-height beta, for a double well in steep tails
    # over the whole range (as in a sampled histogram, whose edges lie far
    # below its peaks, so that no tilt in the bracket makes an edge a peak)
    k1, period, h = 30, 40, 1.0
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k < k1, h - 0.5 * (k1 - k), np.where(k > k1 + period, h - 0.5 * (k - k1 - period), f))
    lnW = -(B0_POTTS8 * E + f)
    assert oracle.interface_tension(POTTS, L, lnW, cnt, B0_POTTS8 - 0.2, B0_POTTS8 + 0.2)[0] == \
        pytest.approx(B0_POTTS8, abs=1e-12)
    with pytest.raises(ValueError):
        oracle.interface_tension(POTTS, L, lnW, cnt, B0_POTTS8 + 0.05, B0_POTTS8 + 0.2)


@pytest.mark.parametrize("model,L,k1,period,lo,hi", [(POTTS, 8, 30, 40, -0.2, 0.2), (POTTS, 12, 60, 80, -0.03, 0.15),
                                                     (POTTS, 12, 60, 80, -0.15, 0.03), (ISING, 8, 20, 30, -0.1, 0.3)])
def test_equal_height_with_a_wide_bracket(model, L, k1, period, lo, hi):
    h = 1.7
    lnW, cnt = double_well(model, L, k1, period, h, B0_POTTS8)
    beta, sigma, ks = oracle.interface_tension(model, L, lnW, cnt, B0_POTTS8 + lo, B0_POTTS8 + hi)
    assert beta == pytest.approx(B0_POTTS8, abs=1e-12)
    assert sigma == pytest.approx(h / L, rel=1e-12)
    assert ks == (k1, k1 + period // 2, k1 + period)


def test_equal_height_ignores_an_isolated_ground_state():
    """The ground state sits alone at k = 0 (k = 1..3 cannot occur) below a
    tail that rises into the ordered peak, as in a sampled Potts histogram.
    Under the tilt of the bracket's upper end it forms a small separate
    maximum; carrying almost no probability, it does not take the split."""
    L = 8
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    k1, period, h = 30, 40, 1.0
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k < k1, h - 0.3 * (k1 - k), np.where(k > k1 + period, h - 0.3 * (k - k1 - period), f))
    f[0] = f[4] - 2.0
    cnt = np.ones(2 * N + 1, np.int64)
    cnt[1:4] = 0
    lnW = -(B0_POTTS8 * E + f)
    beta, sigma, ks = oracle.interface_tension(POTTS, L, lnW, cnt, B0_POTTS8 - 0.05, B0_POTTS8 + 0.05)
    assert beta == pytest.approx(B0_POTTS8, abs=1e-12)
    assert sigma == pytest.approx(h / L, rel=1e-12)
    assert ks == (k1, k1 + period // 2, k1 + period)


def noisy_tail_well(L=8, k1=30, period=40, h=0.5, slope=0.19, dip=5.0):
    """A shallow double well (valley depth 2h, as for a small Potts lattice)
    whose low-energy tail, sampled sparsely, has one bin far below its
    neighbours; the ground state sits alone at k = 0 (k = 1..3 cannot occur)."""
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k < k1, h - slope * (k1 - k), np.where(k > k1 + period, h - 0.3 * (k - k1 - period), f))
    f[9] -= dip
    cnt = np.ones(2 * N + 1, np.int64)
    cnt[1:4] = 0
    return -(B0_POTTS8 * E + f), cnt


def test_equal_height_ignores_a_dip_in_a_sparse_tail():
    """Tilted to the bracket's upper end, the dip is deeper than the phase
    valley and its two sides differ little in height, but the tail side holds
    little probability: the split stays at the phase valley."""
    lnW, cnt = noisy_tail_well()
    beta, sigma, ks = oracle.interface_tension(POTTS, 8, lnW, cnt, B0_POTTS8 - 0.05, B0_POTTS8 + 0.05)
    assert beta == pytest.approx(B0_POTTS8, abs=1e-12)
    assert sigma == pytest.approx(0.5 / 8, rel=1e-12)
    assert ks == (30, 50, 70)
