"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a closed form, an independent
implementation, brute force, or an invariant the method must satisfy, chosen
so that a plausible mistake (a dropped term, a wrong sign or index, a
transposed operand, a wrong boundary) fails at least one of them.
"""
import math
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle
import exact_ising

ISING, POTTS = oracle.ISING, oracle.POTTS


# ------------------------------------------------------------------ Philox

def _torch_philox_binary(tmp_path_factory):
    import torch.utils.cpp_extension as ce
    src = os.path.join(os.path.dirname(__file__), "native", "philox_torch_pin.cpp")
    exe = str(tmp_path_factory.mktemp("ptp") / "ptp")
    inc = []
    for p in ce.include_paths():
        inc += ["-I", p]
    subprocess.check_call(["g++", "-O1", "-std=c++17", *inc, src, "-o", exe])
    return exe


def test_philox_matches_independent_implementation(tmp_path_factory):
    """Philox4x32-10 against PyTorch's header implementation of the same
    published generator (Salmon et al., SC'11), on edge and random counters."""
    exe = _torch_philox_binary(tmp_path_factory)
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6, (1, 2, 3, 4, 5, 6)]
    cases += [tuple(int(v, 16) for v in r[:6]) for r in _kat_rows()]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, 6)) for _ in range(300)]
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = [int(v) for v in oracle.philox(c[:4], c[4:])]
        assert got == ref, (c, got, ref)


def _kat_rows():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    return [line.split() for line in open(path) if line.strip() and not line.startswith("#")]


def test_philox_known_answers():
    """Known-answer rows of the generator (tests/golden; written from memory of
    the authors' published vectors, as the file's header says).  The same
    counters are also run through PyTorch's implementation above, which is the
    pin that does not rest on the file."""
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        assert [int(v) for v in oracle.philox(w[0:4], w[4:6])] == w[6:10], r


def test_philox_output_bits_are_balanced():
    """Every output bit of consecutive counters is 1 about half the time."""
    words = np.array([oracle.philox((i, 7, 3, 0), (1, 0)) for i in range(4096)], np.uint32).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(words.size))


# ------------------------------------------------------------------ exact DOS

def test_bruteforce_ising_L4_equals_kaufman_beale():
    om, _ = oracle.bruteforce(ISING, 2, 4)
    assert list(om) == list(exact_ising.density_of_states(4))


def test_bruteforce_ising_canonical_equals_kaufman():
    """<E> and C_V from summing all 2^16 states equal derivatives of
    Kaufman's ln Z (an independent closed form)."""
    for beta in (0.1, 0.3, 0.4407, 0.6):
        e, e2, _ = oracle.bruteforce_canonical(ISING, 2, 4, beta)
        ek, cvk = exact_ising.kaufman_energy_cv(4, beta)
        assert e / 16 == pytest.approx(ek, rel=1e-9)
        assert beta * beta * (e2 - e * e) / 16 == pytest.approx(cvk, rel=1e-8)


@pytest.mark.parametrize("L", [4, 6, 8])
def test_beale_invariants_and_reachable_mask(L):
    """Exact Omega: total 2^N, symmetric in k <-> 2N-k, Omega(0) = 2,
    Omega(4) = 2N (one flipped spin), Omega(6) = 4N (two adjacent flipped);
    its support is exactly the oracle's reachable mask."""
    N = L * L
    om = np.array([float(v) for v in exact_ising.density_of_states(L)])
    omi = exact_ising.density_of_states(L)
    assert sum(omi) == 2**N
    assert omi[0] == 2 and omi[4] == 2 * N and omi[6] == 4 * N
    assert all(omi[k] == omi[2 * N - k] for k in range(2 * N + 1))
    assert np.array_equal(om > 0, oracle.reachable(ISING, 2, L))


@pytest.fixture(scope="module")
def potts_l3():
    return oracle.bruteforce(POTTS, 8, 3)


def test_bruteforce_potts_L3_closed_forms(potts_l3):
    """8-Potts on the 3x3 torus: total 8^9; Omega(0) = q (uniform states);
    Omega(4) = q(q-1)N (one odd site); Omega(6) = q(q-1)(2N + 2L) (an
    adjacent pair, or a full row/column on the L = 3 torus); Omega(7) =
    q(q-1)(q-2) 2N (an adjacent pair of two different odd colours)."""
    om, _ = potts_l3
    q, N, L = 8, 9, 3
    assert om.sum() == q**N
    assert om[0] == q
    assert om[4] == q * (q - 1) * N
    assert om[6] == q * (q - 1) * (2 * N + 2 * L)
    assert om[7] == q * (q - 1) * (q - 2) * 2 * N
    assert np.array_equal(om > 0, oracle.reachable(POTTS, 8, 3))


def _potts_transfer_matrix_z(q, L, x):
    """sum_k Omega(k) x^k on the L x L torus by a transfer matrix over row
    states (an independent route to the partition function): M[a][b] =
    x^(unsatisfied bonds inside row a + between row a and the row b below),
    and the sum over configurations is Tr(M^L)."""
    import itertools
    rows = np.array(list(itertools.product(range(q), repeat=L)))
    inside = (rows != np.roll(rows, -1, axis=1)).sum(axis=1)
    between = (rows[:, None, :] != rows[None, :, :]).sum(axis=2)
    M = float(x) ** (inside[:, None] + between).astype(np.float64)
    return float(np.trace(np.linalg.matrix_power(M, L)))


@pytest.mark.parametrize("q,L", [(8, 3), (3, 4)])
def test_bruteforce_potts_equals_transfer_matrix(q, L, potts_l3):
    """Every bin of the enumerated Potts Omega(k): the polynomial
    sum_k Omega(k) x^k has degree 2N, so agreeing with the transfer matrix at
    2N + 1 distinct x fixes all of its coefficients."""
    om = potts_l3[0] if (q, L) == (8, 3) else oracle.bruteforce(POTTS, q, L)[0]
    N = L * L
    for x in np.linspace(0.05, 1.0, 2 * N + 1):
        direct = float(np.polynomial.polynomial.polyval(x, om.astype(np.float64)))
        assert direct == pytest.approx(_potts_transfer_matrix_z(q, L, x), rel=1e-11), (q, L, x)


def test_ising_equals_two_state_potts():
    """The Ising model is the q = 2 Potts model (Sec. 3): both count k the
    same way, so brute-force Omega(k) agrees."""
    om_i, _ = oracle.bruteforce(ISING, 2, 4)
    om_p, _ = oracle.bruteforce(POTTS, 2, 4)
    assert np.array_equal(om_i, om_p)


# ------------------------------------------------------------------ table

def test_table_properties():
    rng = np.random.default_rng(7)
    lnW = np.cumsum(rng.normal(0, 3, 129))
    T = oracle.build_table(lnW)
    n = lnW.size
    for k in range(n):
        for dk in range(-4, 5):
            t = k + dk
            v = int(T[k, dk + 4])
            if t < 0 or t >= n:
                assert v == 0
                continue
            d = lnW[t] - lnW[k]
            if d >= 0:
                assert v == 0xFFFFFFFF
            else:
                p = math.exp(d)
                # floor(2^32 p): within one unit of 2^32 p, never above it
                assert v <= p * 2**32 + 1e-6 and v > p * 2**32 - 1 - 1e-6 or v == 0xFFFFFFFF
    # dk = 0 always accepts
    assert np.all(T[:, 4] == 0xFFFFFFFF)


def test_table_detailed_balance_for_energy_models():
    """Metropolis on the multicanonical ensemble (Eq. 1): for every move k ->
    k + dk and its reverse, one direction always accepts and the ratio of the
    two acceptance probabilities is W(k + dk) / W(k) = e^(lnW[k+dk] - lnW[k]),
    up to the quantisation of thresholds in units of 2^-32 (weight
    differences up to 12 here, so the smaller threshold is at least 2^14)."""
    rng = np.random.default_rng(17)
    lnW = np.cumsum(rng.uniform(-3.0, 3.0, 257))
    T = oracle.build_table(lnW).astype(np.float64)
    n = lnW.size
    checked = 0
    for k in range(n):
        for dk in range(1, 5):
            t = k + dk
            if t >= n:
                continue
            fwd, rev = T[k, dk + 4], T[t, -dk + 4]
            assert max(fwd, rev) == 0xFFFFFFFF
            # a threshold T accepts with probability T / 2^32; 0xFFFFFFFF always
            pf = 1.0 if fwd == 0xFFFFFFFF else fwd / 2.0**32
            pr = 1.0 if rev == 0xFFFFFFFF else rev / 2.0**32
            d = lnW[t] - lnW[k]
            assert pf / pr == pytest.approx(math.exp(d), rel=2.0 ** -13), (k, dk)
            checked += 1
    assert checked == 4 * n - 10


def test_table_monotone_in_weight_difference():
    d = np.linspace(-30, 1, 4001)
    lnW = np.stack([np.zeros_like(d), d], axis=1)
    vals = []
    for row in lnW:
        T = oracle.build_table(row)
        vals.append(int(T[0, 5]))
    assert all(a <= b for a, b in zip(vals, vals[1:]))
    assert vals[0] == 0 and vals[-1] == 0xFFFFFFFF


# ------------------------------------------------------------------ flatness

def test_flatness_on_hand_made_histograms():
    """Hand-made histograms over a mask with unreachable holes.  Default rule:
    every reachable bin visited and min/max >= 1/2 (equality counts as flat).
    The paper's rule (Sec. 3): every reachable entry within [avg/2, 2 avg].
    Unreachable bins never count, visited or not."""
    mask = np.array([1, 0, 1, 1, 1, 0, 1, 1], bool)
    h = np.array([10, 0, 5, 7, 9, 0, 6, 10], np.int64)       # min/max = 5/10 exactly
    f = oracle.flatness(h, mask)
    assert f.covered and f.flat and f.min_over_max == 0.5
    assert (f.k_lo, f.k_hi, f.visited, f.reachable) == (0, 7, 6, 6)
    assert f.min_over_avg == pytest.approx(5 / 7.833333333333333)
    h2 = h.copy()
    h2[2] = 4                                                 # 4/10 < 1/2
    assert oracle.flatness(h2, mask).covered and not oracle.flatness(h2, mask).flat
    h3 = h.copy()
    h3[6] = 0                                                 # a reachable bin never visited
    f3 = oracle.flatness(h3, mask)
    assert not f3.covered and not f3.flat and f3.visited == 5
    assert not oracle.flatness(h3, mask, rule=1).flat
    h4 = h.copy()
    h4[5] = 1000                                              # unreachable bins are ignored
    assert oracle.flatness(h4, mask).flat and oracle.flatness(h4, mask).min_over_max == 0.5
    # the paper's rule: avg = 2, min = avg/2 and max = 3 <= 2 avg: flat by it,
    # not by min/max = 1/3; min below avg/2 or max above 2 avg is not flat
    m = np.ones(10, bool)
    p = np.array([1, 2, 2, 2, 2, 2, 2, 2, 2, 3], np.int64)
    assert oracle.flatness(p, m, rule=1).flat and not oracle.flatness(p, m).flat
    assert not oracle.flatness(np.array([1, 3, 3, 3, 3, 3, 3, 3, 3, 3]), m, rule=1).flat   # 1 < 2.8/2
    assert not oracle.flatness(np.array([9, 2, 2, 2, 2, 2, 2, 2, 2, 2]), m, rule=1).flat   # 9 > 2 * 2.7


def test_flatness_rules_are_scale_free_and_nested():
    """Neither rule changes when every count is multiplied by a constant, and
    min/max >= 1/2 implies the paper's rule (min >= max/2 >= avg/2 and
    max <= 2 min <= 2 avg)."""
    rng = np.random.default_rng(8)
    mask = oracle.reachable(ISING, 2, 8)
    n_flat = 0
    for _ in range(400):
        h = np.where(mask, rng.integers(1, 40, mask.size) + rng.integers(30, 60), 0).astype(np.int64)
        for rule in (0, 1):
            assert oracle.flatness(h, mask, rule=rule).flat == oracle.flatness(7 * h, mask, rule=rule).flat
        if oracle.flatness(h, mask).flat:
            n_flat += 1
            assert oracle.flatness(h, mask, rule=1).flat
    assert 0 < n_flat < 400


# ------------------------------------------------------------------ sampler

@pytest.mark.parametrize("model,L,q", [(ISING, 4, 2), (ISING, 6, 2), (POTTS, 3, 8), (POTTS, 5, 8)])
def test_tracked_state_and_histogram_invariants(model, L, q):
    """Tracked k and M equal a full recompute from the spins; each chain
    adds exactly one count per recorded sweep; unreachable bins stay empty."""
    r = oracle.OracleRun(model, L, 37, 99, q=q, n_threads=3)
    rng = np.random.default_rng(1)
    r.set_log_weights(np.cumsum(rng.normal(0, 0.7, r.n_bins)))
    r.sweeps(5, oracle.REC_NONE)
    r.hist[:] = 0
    r.sweeps(40, oracle.REC_MUCA)
    for c in range(r.n_chains):
        k, m = oracle.energy(model, L, r.spins[c])
        assert (k, m) == (r.k[c], r.m[c])
    assert np.all(r.hist.sum(axis=1) == 40)
    assert np.all(r.merged()[~r.mask] == 0)
    assert np.all(r.spins < q)


@pytest.mark.parametrize("model,q", [(ISING, 2), (POTTS, 8)])
def test_infinite_temperature_moves(model, q):
    """With lnW = 0 every move is accepted: after one sweep every site has
    changed, and the Potts offset (s' - s - 1) mod q is uniform on 0..q-2."""
    r = oracle.OracleRun(model, 6, 400, 5, q=q)
    before = r.spins.copy()
    r.sweeps(1, oracle.REC_NONE)
    assert np.all(r.spins != before)
    if model == POTTS:
        off = ((r.spins.astype(int) - before.astype(int) - 1) % q).ravel()
        assert off.max() == q - 2
        cnt = np.bincount(off, minlength=q - 1)
        assert stats.chisquare(cnt).pvalue > 1e-3


def test_initial_spins_are_uniform():
    r = oracle.OracleRun(POTTS, 16, 64, 3, q=8)
    cnt = np.bincount(r.spins.ravel(), minlength=8)
    assert stats.chisquare(cnt).pvalue > 1e-3
    r = oracle.OracleRun(ISING, 16, 64, 3)
    assert abs(r.spins.mean() - 0.5) < 5 * 0.5 / math.sqrt(r.spins.size)


def _chisq(obs, exp_p):
    n = obs.sum()
    e = exp_p * n
    keep = e >= 5
    o2 = np.append(obs[keep], obs[~keep].sum())
    e2 = np.append(e[keep], e[~keep].sum())
    if e2[-1] == 0:
        o2, e2 = o2[:-1], e2[:-1]
    return stats.chisquare(o2, e2).pvalue


@pytest.mark.parametrize("model,L,q,beta", [(ISING, 4, 2, 0.3), (ISING, 4, 2, 0.45), (POTTS, 3, 8, 1.0)])
def test_canonical_limit_chi_square(model, L, q, beta, potts_l3):
    """lnW = -beta E turns the multicanonical chain into canonical Metropolis,
    Eq. (1) with W = exp(-beta E).  One end-of-run sample per chain (chains
    are independent) must follow Omega(E) exp(-beta E) / Z exactly."""
    if model == ISING:
        om, _ = oracle.bruteforce(ISING, 2, L)
    else:
        om, _ = potts_l3
    E = oracle.energies(model, L)
    r = oracle.OracleRun(model, L, 20000, 11, q=q)
    r.set_log_weights(-beta * E)
    r.sweeps(40, oracle.REC_NONE)
    r.hist[:] = 0
    r.sweeps(1, oracle.REC_MUCA)
    obs = r.merged().astype(np.float64)
    w = om * np.exp(-beta * (E - E.min()))
    p = w / w.sum()
    assert _chisq(obs, p) > 1e-3


def test_muca_converges_to_exact_dos_ising_L4():
    """Iterating W <- W/H to a flat histogram gives lnW = -ln Omega + const
    (Sec. 2: W = 1/Omega makes every energy equally likely)."""
    r = oracle.OracleRun(ISING, 4, 64, 21)
    flat = False
    for _ in range(40):
        _, fl, _ = r.iterate(2000)
        flat = flat or fl.flat
    assert flat
    lo = np.log(np.array(exact_ising.density_of_states(4), np.float64), where=r.mask,
                out=np.full(r.n_bins, -np.inf))
    d = (-r.lnW - lo)[r.mask]
    d -= d.mean()
    assert np.abs(d).max() < 0.1


def test_muca_converges_to_exact_dos_potts_L3(potts_l3):
    om, _ = potts_l3
    r = oracle.OracleRun(POTTS, 3, 64, 22, q=8)
    flat = False
    for _ in range(40):
        _, fl, _ = r.iterate(2000)
        flat = flat or fl.flat
    assert flat
    lo = np.log(om.astype(np.float64), where=r.mask, out=np.full(r.n_bins, -np.inf))
    d = (-r.lnW - lo)[r.mask]
    d -= d.mean()
    assert np.abs(d).max() < 0.15


def test_small_ising_run_reaches_exact_dos_L8():
    """The Ising L = 8 run with 4 chains and 20 iterations of 1e4 sweeps
    becomes flat and its weights match Beale's exact ln Omega."""
    r = oracle.OracleRun(ISING, 8, 4, 1)
    flats = []
    for _ in range(20):
        _, fl, _ = r.iterate(10_000)
        flats.append(fl.flat)
    assert flats[-1] and sum(flats) >= 8
    lo = exact_ising.log_dos(8)
    d = (-r.lnW - lo)[r.mask]
    d -= d.mean()
    assert np.abs(d).max() < 0.35 and d.std() < 0.1


def _norm_update(H, lnW):
    out = np.array(lnW, np.float64)
    oracle.lib().orc_recursion_norm(H.size, np.ascontiguousarray(H, np.int64), out)
    return out


def test_normalized_recursion_hand_example():
    """The update shifted to zero mean over the visited bins (a reading of
    Sec. 2 that fixes W / H's free constant), worked by hand: H = (0, 4, 1, 16)
    has ln H = (ln 4, 0, ln 16) on its visited bins, mean ln 4, so the weights
    move by (0, 0, +ln 4, -ln 4)."""
    H = np.array([0, 4, 1, 16], np.int64)
    got = _norm_update(H, [0.5, 0.0, 0.0, 0.0])
    assert got == pytest.approx([0.5, 0.0, math.log(4), -math.log(4)], abs=1e-15)
    # the plain recursion on the same counts: (0.5, -ln 4, 0, -ln 16)
    plain = np.array([0.5, 0.0, 0.0, 0.0])
    oracle.lib().orc_recursion(4, H, plain)
    assert plain == pytest.approx([0.5, -math.log(4), 0.0, -math.log(16)], abs=1e-15)


def test_normalized_recursion_properties():
    """Unvisited bins keep their weights; over the visited bins the change
    has zero mean and differs from the plain recursion's by one constant; the
    result does not depend on how the histogram is normalized (H and 64 H give
    the same weights), which the plain recursion's does; a flat histogram
    leaves the weights unchanged."""
    rng = np.random.default_rng(5)
    n = 301
    H = rng.integers(1, 5000, n).astype(np.int64)
    H[rng.random(n) < 0.3] = 0
    lnW = rng.normal(0, 3, n)
    got = _norm_update(H, lnW)
    vis = H > 0
    assert np.array_equal(got[~vis], lnW[~vis])
    delta = got[vis] - lnW[vis]
    assert abs(delta.mean()) < 1e-12
    plain = lnW.copy()
    oracle.lib().orc_recursion(n, H, plain)
    shift = (got - plain)[vis]
    assert np.ptp(shift) < 1e-12 and shift[0] == pytest.approx(np.log(H[vis]).mean(), rel=1e-12)
    assert _norm_update(64 * H, lnW) == pytest.approx(got, abs=1e-12)
    plain64 = lnW.copy()
    oracle.lib().orc_recursion(n, 64 * H, plain64)
    assert not np.allclose(plain64[vis], plain[vis])
    flat = np.where(vis, 777, 0).astype(np.int64)
    assert _norm_update(flat, lnW) == pytest.approx(lnW, abs=1e-12)


def test_correction_function_properties():
    """The correction function (Sec. 3) leaves the sampled region alone, puts
    every reachable bin outside it on the line through the edge bin and the
    bin L reachable bins inward, and is the identity on weights that are
    already linear in k."""
    L = 6
    mask = oracle.reachable(ISING, 2, L)
    n = mask.size
    H = np.zeros(n, np.int64)
    H[20:41:2] = 5                      # sampled region k = 20..40
    rng = np.random.default_rng(2)
    lnW = rng.normal(0, 3, n)
    before = lnW.copy()
    oracle.correction(lnW, H, mask, L)
    assert np.array_equal(lnW[20:41], before[20:41])
    # lower edge: anchor 20 and the bin 6 reachable bins inward, k = 32
    s = (before[20] - before[32]) / (20 - 32)
    for k in range(0, 20):
        if mask[k]:
            assert lnW[k] == pytest.approx(before[20] + s * (k - 20), abs=1e-12)
        else:
            assert lnW[k] == before[k]
    s = (before[40] - before[28]) / (40 - 28)
    for k in range(41, n):
        if mask[k]:
            assert lnW[k] == pytest.approx(before[40] + s * (k - 40), abs=1e-12)
    lin = 0.37 * np.arange(n) - 4.0
    lin2 = lin.copy()
    oracle.correction(lin2, H, mask, L)
    assert np.allclose(lin2, lin, atol=1e-12)
