"""Pins of the oracle's time-series reweighting, Eq. (2), grouped by bin."""
import numpy as np
import pytest

import oracle
import exact_ising

ISING = oracle.ISING


@pytest.mark.parametrize("L", [4, 8])
def test_reweighting_exact_weights_gives_kaufman(L):
    """With W = 1/Omega (the converged multicanonical weights, Sec. 2) and the
    same count in every reachable bin, Eq. (2) reduces to the canonical
    average over the exact density of states; compare with derivatives of
    Kaufman's closed-form ln Z."""
    om = exact_ising.density_of_states(L)
    lnom = exact_ising.log_dos(L)
    mask = np.array([v > 0 for v in om])
    lnW = np.where(mask, -lnom, 0.0)
    cnt = np.where(mask, 1000, 0).astype(np.int64)
    sabs = np.zeros_like(cnt)
    betas = [0.3, 0.4, 0.4407, 0.5, 0.6]
    e, cv, _ = oracle.reweight(ISING, L, lnW, cnt, sabs, betas)
    for b, ei, ci in zip(betas, e, cv):
        ek, ck = exact_ising.kaufman_energy_cv(L, b)
        assert ei == pytest.approx(ek, rel=1e-11)
        assert ci == pytest.approx(ck, rel=1e-9)


def test_reweighting_magnetization_matches_state_sum():
    """With lnW = 0, counts = Omega and |M| sums from enumeration, Eq. (2)
    gives the canonical <|M|>; compare with a direct sum over all states."""
    om, sm = oracle.bruteforce(ISING, 2, 4)
    lnW = np.zeros(om.size)
    for b in (0.2, 0.44, 0.7):
        e, cv, am = oracle.reweight(ISING, 4, lnW, om, sm, [b])
        ee, ee2, aam = oracle.bruteforce_canonical(ISING, 2, 4, b)
        assert e[0] == pytest.approx(ee / 16, rel=1e-12)
        assert cv[0] == pytest.approx(b * b * (ee2 - ee * ee) / 16, rel=1e-9)
        assert am[0] == pytest.approx(aam / 16, rel=1e-12)


def test_production_run_reweights_to_exact_L4():
    """A full run at Ising L = 4 (weights to flatness, re-thermalisation,
    production, Sec. 3 and 5) reproduces the exact <E> and C_V within a few
    per cent over beta in [0.3, 0.6]."""
    r = oracle.OracleRun(ISING, 4, 64, 5)
    for _ in range(15):
        r.iterate(2000)
    cnt, sab = r.production(500, 5000)
    betas = np.linspace(0.3, 0.6, 7)
    e, cv, am = oracle.reweight(ISING, 4, r.lnW, cnt, sab, betas)
    for b, ei, ci, mi in zip(betas, e, cv, am):
        ek, ck = exact_ising.kaufman_energy_cv(4, b)
        ee, ee2, aam = oracle.bruteforce_canonical(ISING, 2, 4, b)
        assert ei == pytest.approx(ek, rel=0.01)
        assert ci == pytest.approx(ck, rel=0.05)
        assert mi == pytest.approx(aam / 16, rel=0.01)


@pytest.mark.parametrize("q", [3, 4])
def test_potts_reweighting_of_an_ideal_histogram_equals_derivatives_of_ln_z(q):
    """q-state Potts on the 3x3 torus (E = -2N + k).  For any positive counts
    c_k, the weights lnW = ln(c_k / Omega_k) make c the ideal histogram of the
    ensemble Omega W, and Eq. (2) must return the exact canonical averages:
    <E>/N = -d ln Z/d beta / N and C_V = beta^2 d^2 ln Z/d beta^2 / N, with
    ln Z(beta) = ln sum_k Omega_k exp(-beta E_k) differentiated by mpmath.
    Random counts catch a sign slip on lnW or on ln cnt; the energies catch
    an Ising-style 2k."""
    import mpmath
    POTTS = oracle.POTTS
    om, _ = oracle.bruteforce(POTTS, q, 3)
    N = 9
    mask = om > 0
    rng = np.random.default_rng(q)
    c = np.where(mask, rng.integers(1, 500, om.size), 0).astype(np.int64)
    lnW = np.where(mask, np.log(np.maximum(c, 1)) - np.log(np.maximum(om, 1).astype(np.float64)), 0.0)
    betas = [0.2, 0.9, 1.3, 2.0]
    e, cv, _ = oracle.reweight(POTTS, 3, lnW, c, np.zeros_like(c), betas)
    mpmath.mp.dps = 40
    ks = [int(k) for k in np.nonzero(mask)[0]]

    def lnz(b):
        return mpmath.log(mpmath.fsum(int(om[k]) * mpmath.exp(-b * (-2 * N + k)) for k in ks))

    for b, ei, ci in zip(betas, e, cv):
        d1 = mpmath.diff(lnz, mpmath.mpf(b))
        d2 = mpmath.diff(lnz, mpmath.mpf(b), 2)
        assert ei == pytest.approx(float(-d1 / N), rel=1e-12)
        assert ci == pytest.approx(float(b * b * d2 / N), rel=1e-10)
