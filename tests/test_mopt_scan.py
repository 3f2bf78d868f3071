"""Host logic of the M_opt scan (Sec. 4, Eq. 5): the descending scan over
sweeps per iteration, its work cap and its stopping rule, on a synthetic
N_iter(M) with a known minimum of N_iter M p."""
import math

import pytest

import paper_1212_3975_amd.mopt_scan as ms

SWEEPS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024]


def synthetic(m_star, n_floor=6):
    """N_iter(M): a floor of n_floor iterations above M*, growing as (M*/M)^2
    below it; N_iter M is then minimal at M*."""
    calls = []

    def n_iter(model, L, p, M, seed, cap, launch):
        calls.append((p, M, seed, cap))
        n = n_floor + seed % 2 if M >= m_star else math.ceil(n_floor * (m_star / M) ** 2)
        return n if n <= cap else None
    return n_iter, calls


@pytest.mark.parametrize("m_star", [4, 64, 256])
def test_descending_scan_finds_the_minimum(monkeypatch, m_star):
    fn, calls = synthetic(m_star)
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    best, recs = ms.scan_p("ising", 16, 64, SWEEPS, 4, 400, 1e12, {}, lambda r: None)
    assert best["M"] == m_star and not best["upper_edge"]
    assert best["mean_n_iter"] == pytest.approx(6.5)
    assert best["total_sweeps"] == pytest.approx(6.5 * m_star * 64)
    # below M* the total N_iter M p doubles per halving of M: 1.85 x the best
    # at M*/2, past twice the best at M*/4, where the scan stops
    assert [r["M"] for r in recs] == [M for M in SWEEPS[::-1] if M >= m_star // 4]


def test_work_cap_bounds_each_run_and_flags_the_upper_edge(monkeypatch):
    fn, calls = synthetic(2048)
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    p, max_total = 64, 5e6
    best, recs = ms.scan_p("ising", 16, p, SWEEPS, 3, 400, max_total, {}, lambda r: None)
    for (_, M, _, cap) in calls:
        assert cap * M * p <= max_total and cap <= 400
    # every M is below M*: the largest scanned is the best, at the edge
    assert best["M"] == 1024 and best["upper_edge"]


def test_a_seed_beyond_seeds_times_the_best_stops_the_scan(monkeypatch):
    def fn(model, L, p, M, seed, cap, launch):
        n = {1024: 4, 512: 6, 256: 40}.get(M, 10 ** 6)
        return n if n <= cap else None
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    best, recs = ms.scan_p("ising", 16, 8, SWEEPS, 5, 400, 1e12, {}, lambda r: None)
    assert best["M"] == 512 and best["total_sweeps"] == 6 * 512 * 8
    last = recs[-1]
    # at M = 256 one seed may spend 5 x the best total: 5 * 6 * 512 / 256 = 60
    assert last["M"] == 256 and last["iteration_cap"] == 60
    assert "mean_n_iter" in last and last["total_sweeps"] > 2 * best["total_sweeps"]
    assert len(recs) == 3


def test_an_unconverged_seed_ends_the_scan_without_the_rest(monkeypatch):
    fn, calls = synthetic(64)
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    best, recs = ms.scan_p("ising", 16, 64, [16, 32, 64], 5, 30, 1e12, {}, lambda r: None)
    assert best["M"] == 64
    # M = 32 needs 24 iterations, within the cap of 30; M = 16 needs 96, and
    # its first seed ends the scan
    assert [r["M"] for r in recs] == [64, 32, 16]
    assert recs[-1]["n_iter"] == [None] and recs[-1]["converged"] == 0
    assert [c[1] for c in calls].count(16) == 1


def test_fit_of_m1_with_slope_minus_one():
    assert ms.fit_m1([64, 256, 1024], [256, 64, 16]) == pytest.approx(16384)


def test_a_top_m_cut_by_the_work_cap_does_not_end_the_scan(monkeypatch):
    fn, calls = synthetic(64, n_floor=8)
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    # at M = 1024 and 512 the work cap allows 7 and 15 iterations: the first
    # run fails (8 needed), the scan goes on
    best, recs = ms.scan_p("ising", 16, 64, SWEEPS, 2, 400, 5e5, {}, lambda r: None)
    assert recs[0]["M"] == 1024 and recs[0]["converged"] == 0 and recs[0]["iteration_cap"] == 7
    assert best["M"] == 64 and not best["upper_edge"]


def test_an_iteration_cap_failure_before_any_success_ends_the_scan(monkeypatch):
    fn, calls = synthetic(4096)
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    best, recs = ms.scan_p("ising", 16, 64, SWEEPS, 3, 20, 1e12, {}, lambda r: None)
    assert best is None and len(recs) == 1 and recs[0]["n_iter"] == [None]


def test_cap_bound_flags_an_iteration_cap_below_the_best(monkeypatch):
    def fn(model, L, p, M, seed, cap, launch):
        n = {64: 20, 32: 45, 16: 60}.get(M, 10 ** 6)
        return n if n <= cap else None
    monkeypatch.setattr(ms, "iterations_to_flat", fn)
    best, _ = ms.scan_p("ising", 16, 8, [16, 32, 64], 2, 50, 1e12, {}, lambda r: None)
    # M = 16 failed at 50 iterations: 50 * 16 * 8 = 6400 < best 20 * 64 * 8
    assert best["M"] == 64 and best["cap_bound"]
    # with a larger cap, M = 16 converges (60 * 16 * 8 = 7680) and is the best
    best, _ = ms.scan_p("ising", 16, 8, [16, 32, 64], 2, 1000, 1e12, {}, lambda r: None)
    assert best["M"] == 16 and not best["cap_bound"]
