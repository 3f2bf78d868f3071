"""Pins of the oracle's multimagnetic Ising ensemble (Sec. 4): weights W(M)
over the magnetization at a fixed inverse temperature beta, acceptance
min(1, exp(-beta dE) W(M') / W(M)).

- beta = 0 and flat weights accept every flip: one sequential sweep
  complements the lattice.
- Flat weights at beta > 0 leave the canonical ensemble: the sampled P(m) and
  the mean bond count per m must match the exact values from enumerating all
  2^16 states of the L = 4 lattice.  A wrong sign of beta, a missing factor 2
  in dE = 2 dk, or a mislabelled column fails this.
- Iterated weights converge to -ln P_beta(m) up to a constant (flat histogram
  over m).
- Every threshold pairs with the reverse move (m' back to m, -dk): at least
  one of the two is "always", the other is the threshold of -|delta|
  (detailed balance of the table)."""
import math

import numpy as np
import pytest

import oracle
from oracle import ISING_MAG

BETA0 = 0.5 * math.log(1.0 + math.sqrt(2.0))   # Sec. 3: Ising transition point


def test_beta_zero_flat_weights_complement_the_lattice():
    orc = oracle.OracleRun(ISING_MAG, 6, 5, seed=3, beta=0.0)
    s0, k0, m0 = orc.spins.copy(), orc.k.copy(), orc.m.copy()
    assert np.all(orc.T == 0xFFFFFFFF) or np.all((orc.T == 0xFFFFFFFF) | (orc.T == 0))
    orc.sweeps(1, oracle.REC_NONE)
    assert np.array_equal(orc.spins, 1 - s0)
    assert np.array_equal(orc.k, k0) and np.array_equal(orc.m, -m0)


def test_table_detailed_balance():
    L, beta = 6, 0.61
    N = L * L
    rng = np.random.default_rng(2)
    lnW = np.cumsum(rng.normal(0.0, 0.7, N + 1))
    T = oracle.build_table_mag(L, beta, lnW)
    sat = 0xFFFFFFFF
    checked = 0
    for m in range(N + 1):
        for u in (0, 1):
            mp = m - 1 if u else m + 1
            for j in range(5):
                t = int(T[m, j + 5 * u])
                if not 0 <= mp <= N:
                    assert t == 0
                    continue
                # the reverse move: from m' flip the same spin back (the other
                # value), with the neighbours unchanged: dk -> -dk, j -> 4 - j
                r = int(T[mp, (4 - j) + 5 * (1 - u)])
                assert t == sat or r == sat
                dk = 2 * j - 4
                delta = (lnW[mp] - lnW[m]) - beta * 2.0 * dk
                small = min(t, r)
                if small != sat:
                    expect = math.floor(math.ldexp(math.exp(-abs(delta)), 32))
                    assert abs(small - expect) <= 1
                checked += 1
    assert checked == 2 * 5 * N


@pytest.mark.parametrize("beta", [0.3, BETA0])
def test_flat_weights_sample_the_canonical_magnetization(beta):
    L, chains, n_prod = 4, 256, 3000
    orc = oracle.OracleRun(ISING_MAG, L, chains, seed=11, beta=beta)
    cnt, ksum = orc.production(300, n_prod)
    n = cnt.sum()
    assert n == chains * n_prod
    p_exact, k_exact = oracle.bruteforce_mag(L, beta)
    p_emp = cnt / n
    # chains are independent, sweeps within a chain correlated: allow an
    # autocorrelation time of 10 sweeps in the binomial error
    err = np.sqrt(p_exact * (1 - p_exact) * 10.0 / n) + 1e-4
    assert np.all(np.abs(p_emp - p_exact) < 6 * err), (p_emp, p_exact)
    sel = cnt > 2000
    k_emp = ksum[sel] / cnt[sel]
    assert np.all(np.abs(k_emp - k_exact[sel]) < 0.15 * np.sqrt(k_exact[sel] + 1.0)), (k_emp, k_exact[sel])


def test_iterated_weights_converge_to_minus_log_p():
    L, beta = 4, 1.5 * BETA0
    N = L * L
    orc = oracle.OracleRun(ISING_MAG, L, 64, seed=5, beta=beta)
    for it in range(60):
        H, fl, _ = orc.iterate(2000)
        if fl.flat and it > 8:
            break
    assert fl.flat
    p_exact, _ = oracle.bruteforce_mag(L, beta)
    # W ~ 1/P: lnW(m) + ln P(m) is constant over m (the statistical error of
    # the weights is a few per cent at this length)
    c = orc.lnW + np.log(p_exact)
    assert np.ptp(c) < 0.25, c
    # the two ordered peaks are far more likely than M = 0 at 1.5 beta_0
    assert p_exact[0] / p_exact[N // 2] > 10.0


def _ising_omega_k_m(L):
    """Omega(k, m) of the L x L Ising torus (k unsatisfied bonds, m up spins)
    by a transfer matrix over row states: the rows of a configuration form a
    cycle a_0 .. a_{L-1}, each row contributes its own unsatisfied bonds, the
    bonds to the row below and its up spins.  Polynomials in (x^k, y^m) are
    carried as count arrays.  Independent of the oracle's enumeration."""
    import itertools
    N = L * L
    rows = np.array(list(itertools.product((0, 1), repeat=L)))
    inside = (rows != np.roll(rows, -1, axis=1)).sum(axis=1)
    between = (rows[:, None, :] != rows[None, :, :]).sum(axis=2)
    ups = rows.sum(axis=1)
    S = rows.shape[0]
    total = np.zeros((2 * N + 1, N + 1))
    for a0 in range(S):
        vec = np.zeros((S, 2 * N + 1, N + 1))
        vec[a0, 0, 0] = 1.0
        for step in range(L):
            new = np.zeros_like(vec)
            for a in range(S):
                if not vec[a].any():
                    continue
                for b in range(S):
                    if step == L - 1 and b != a0:
                        continue
                    dk, dm = inside[a] + between[a, b], ups[a]
                    new[b, dk:, dm:] += vec[a, :2 * N + 1 - dk, :N + 1 - dm]
            vec = new
        total += vec[a0]
    return total


@pytest.mark.parametrize("beta", [0.3, 0.66])
def test_bruteforce_mag_equals_transfer_matrix(beta):
    """The enumerated canonical P(m) and mean k per m of L = 4 equal those of
    the transfer matrix; summed over m, its Omega(k) is Beale's."""
    import exact_ising
    L = 4
    om = _ising_omega_k_m(L)
    assert om.sum() == 2 ** 16
    assert list(om.sum(axis=1).astype(np.int64)) == [int(v) for v in exact_ising.density_of_states(L)]
    k = np.arange(om.shape[0])[:, None]
    w = om * np.exp(-2.0 * beta * k)             # e^{-beta E} with E = -2N + 2k, up to a constant
    p_tm = w.sum(axis=0) / w.sum()
    km_tm = (w * k).sum(axis=0) / w.sum(axis=0)
    p, km = oracle.bruteforce_mag(L, beta)
    # the enumeration sums 2^16 weights in another order: agreement to rounding
    np.testing.assert_allclose(p, p_tm, rtol=1e-10)
    np.testing.assert_allclose(km, km_tm, rtol=1e-10)
