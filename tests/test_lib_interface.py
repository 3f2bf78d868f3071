"""The library's host implementation of the interface-tension analysis
(mucaEqualHeight, Sec. 5, Eq. 9; no GPU needed) against the oracle, on the
closed-form double wells of test_oracle_interface and on noisy counts."""
import numpy as np
import pytest

import oracle
from oracle import POTTS
from test_oracle_interface import B0_POTTS8, double_well, noisy_tail_well


def _lib_vs_oracle(model, L, lnW, cnt, blo, bhi):
    import paper_1212_3975_amd as pm
    got = pm.equal_height(model, L, lnW, cnt, blo, bhi)
    beta, sigma, ks = oracle.interface_tension(model, L, lnW, cnt, blo, bhi)
    assert got["beta"] == pytest.approx(beta, rel=1e-12, abs=1e-12)
    assert got["sigma"] == pytest.approx(sigma, rel=1e-10, abs=1e-13)
    assert got["k_peaks"] == ks
    kk, a = oracle._log_canonical(model, L, lnW, cnt, got["beta"])
    ref = a - (a.max() + np.log(np.exp(a - a.max()).sum()))
    np.testing.assert_allclose(got["lnP"][kk], ref, rtol=0, atol=1e-11)
    assert np.all(np.isneginf(got["lnP"][cnt == 0]))
    return got


@pytest.mark.parametrize("tilt", [0.0, 0.05])
def test_library_equal_height_matches_oracle(tilt):
    rng = np.random.default_rng(11)
    L = 12
    N = L * L
    lnW, cnt = double_well(POTTS, L, 60, 80, 2.2, B0_POTTS8 + tilt)
    _lib_vs_oracle(POTTS, L, lnW, cnt, B0_POTTS8 + tilt - 0.02, B0_POTTS8 + tilt + 0.015)
    # Poisson noise on the counts: ties and ragged peaks, same answer on both sides
    noisy = rng.poisson(np.where(cnt > 0, 400.0, 0.0)).astype(np.int64)
    noisy[(cnt > 0) & (noisy == 0)] = 1
    _lib_vs_oracle(POTTS, L, lnW, noisy, B0_POTTS8 + tilt - 0.02, B0_POTTS8 + tilt + 0.015)
    assert N > 0


def test_library_equal_height_errors():
    import paper_1212_3975_amd as pm
    L = 8
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    # a double well with steep flanks over the whole range; in a bracket above
    # its equal-height beta the peaks neither cross nor show a balanced valley
    k1, period, h = 30, 40, 1.0
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k < k1, h - 0.5 * (k1 - k), np.where(k > k1 + period, h - 0.5 * (k - k1 - period), f))
    lnW, cnt = -(B0_POTTS8 * E + f), np.ones(2 * N + 1, np.int64)
    with pytest.raises(pm.MucaError, match="do not cross|no two peaks"):
        pm.equal_height(POTTS, L, lnW, cnt, B0_POTTS8 + 0.05, B0_POTTS8 + 0.2)
    one = -(B0_POTTS8 * E - 0.01 * (k - 60.0) ** 2)   # one peak
    with pytest.raises(pm.MucaError, match="no two peaks"):
        pm.equal_height(POTTS, L, one, cnt, B0_POTTS8 - 0.2, B0_POTTS8 + 0.2)
    with pytest.raises(pm.MucaError, match="2N\\+1"):
        pm.equal_height(POTTS, L, lnW[:-1], cnt[:-1], 1.0, 1.5)
    with pytest.raises(pm.MucaError):
        pm.equal_height(POTTS, L, lnW, cnt, 1.5, 1.0)


def test_library_equal_height_long_tail():
    L, k1, period, h, tail = 12, 60, 80, 1.9, 100
    N = L * L
    E = oracle.energies(POTTS, L)
    k = np.arange(2 * N + 1)
    lo, hi = k1 - period // 2 + 1, k1 + period + period // 2 - 1
    f = h * np.cos(2.0 * np.pi * (k - k1) / period)
    f = np.where(k > hi, f[hi] - 0.05 * (k - hi), f)
    cnt = np.zeros(2 * N + 1, np.int64)
    cnt[lo:hi + tail + 1] = 1
    got = _lib_vs_oracle(POTTS, L, -(B0_POTTS8 * E + f), cnt, B0_POTTS8 - 0.02, B0_POTTS8 + 0.015)
    assert got["sigma"] == pytest.approx(h / L, rel=1e-12)


def test_library_equal_height_refuses_the_magnetization_axis():
    import paper_1212_3975_amd as pm
    L = 8
    lnW, cnt = double_well(POTTS, L, 30, 40, 1.0, B0_POTTS8)
    with pytest.raises(pm.MucaError):
        pm.equal_height(pm.ISING_MAG, L, lnW, cnt, 1.3, 1.4)


@pytest.mark.parametrize("lo,hi", [(-0.03, 0.15), (-0.15, 0.03), (-0.2, 0.2)])
def test_library_equal_height_wide_bracket_matches_oracle(lo, hi):
    """Brackets where one phase dominates over most of the range: the split at
    the valley keeps both sides on the true crossing, clean and noisy."""
    rng = np.random.default_rng(13)
    L = 12
    lnW, cnt = double_well(POTTS, L, 60, 80, 1.7, B0_POTTS8)
    got = _lib_vs_oracle(POTTS, L, lnW, cnt, B0_POTTS8 + lo, B0_POTTS8 + hi)
    assert got["beta"] == pytest.approx(B0_POTTS8, abs=1e-12)
    noisy = rng.poisson(np.where(cnt > 0, 400.0, 0.0)).astype(np.int64)
    noisy[(cnt > 0) & (noisy == 0)] = 1
    got = _lib_vs_oracle(POTTS, L, lnW, noisy, B0_POTTS8 + lo, B0_POTTS8 + hi)
    assert abs(got["beta"] - B0_POTTS8) < 2e-3


def test_library_equal_height_sparse_tail_matches_oracle():
    lnW, cnt = noisy_tail_well()
    got = _lib_vs_oracle(POTTS, 8, lnW, cnt, B0_POTTS8 - 0.05, B0_POTTS8 + 0.05)
    assert got["k_peaks"] == (30, 50, 70)
