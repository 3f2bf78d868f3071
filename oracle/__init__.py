"""CPU oracle for parallel multicanonical sampling -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls it and shares no code
with it.

The sampler, table and recursion are plain C loops (``muca_oracle.c``); this
module wraps them with ctypes and adds, in plain numpy:
  - the flatness test of the weight iteration (Sec. 3: full range covered and
    every entry within bounds of the others);
  - the correction function (Sec. 3), which continues lnW linearly beyond the
    sampled region after a recursion;
  - time-series reweighting, Eq. (2), written over energy bins;
  - the interface tension of Eq. (9) from the equal-height reweighted
    energy histogram (Sec. 5).
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import build as _build

ISING, POTTS, ISING_MAG = 0, 1, 2
REC_NONE, REC_MUCA, REC_PROD = 0, 1, 2
TCOLS = 9
TCOLS_MAG = 10

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        c_int, c_u64, c_u32, c_dbl = ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_energy.argtypes = [c_int, c_int, u8p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.orc_reachable.argtypes = [c_int, c_int, c_int, u8p]
        L.orc_bruteforce.argtypes = [c_int, c_int, c_int, i64p, i64p]
        L.orc_bruteforce_canonical.argtypes = [c_int, c_int, c_int, c_dbl,
                                               ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]
        L.orc_init.argtypes = [c_int, c_int, c_int, c_int, c_int, c_u64, u8p, i32p, i32p]
        L.orc_build_table.argtypes = [c_int, f64p, u32p]
        L.orc_build_table_mag.argtypes = [c_int, c_dbl, f64p, u32p]
        L.orc_bruteforce_mag.argtypes = [c_int, c_dbl, f64p, f64p]
        L.orc_sweeps.argtypes = [c_int, c_int, c_int, c_int, c_int, c_u64, c_u32, c_int, c_int, u32p, u8p,
                                 i32p, i32p, i32p, i64p, c_int]
        L.orc_merge.argtypes = [c_int, c_int, i32p, i64p]
        L.orc_recursion.argtypes = [c_int, i64p, f64p]
        L.orc_recursion_norm.argtypes = [c_int, i64p, f64p]
        for f in ("orc_philox4x32_10", "orc_energy", "orc_reachable", "orc_bruteforce",
                  "orc_bruteforce_canonical", "orc_init", "orc_build_table", "orc_build_table_mag",
                  "orc_bruteforce_mag", "orc_sweeps",
                  "orc_merge", "orc_recursion", "orc_recursion_norm"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ------------------------------------------------------------------ primitives

def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def energy(model: int, L: int, spins: np.ndarray):
    k, m = ctypes.c_int32(), ctypes.c_int32()
    lib().orc_energy(model, L, np.ascontiguousarray(spins, np.uint8), ctypes.byref(k), ctypes.byref(m))
    return k.value, m.value


def n_bins_of(model: int, L: int) -> int:
    """2N+1 energy bins (k = 0..2N), or N+1 magnetization bins (m = number of
    up spins) for the multimagnetic ensemble."""
    return L * L + 1 if model == ISING_MAG else 2 * L * L + 1


def reachable(model: int, q: int, L: int) -> np.ndarray:
    mask = np.zeros(n_bins_of(model, L), np.uint8)
    lib().orc_reachable(model, q, L, mask)
    return mask.astype(bool)


def bruteforce(model: int, q: int, L: int):
    """Exact Omega(k) and sum of |M| per k by enumerating all states."""
    nb = 2 * L * L + 1
    om, sm = np.zeros(nb, np.int64), np.zeros(nb, np.int64)
    lib().orc_bruteforce(model, q, L, om, sm)
    return om, sm


def bruteforce_canonical(model: int, q: int, L: int, beta: float):
    e, e2, am = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_bruteforce_canonical(model, q, L, beta, ctypes.byref(e), ctypes.byref(e2), ctypes.byref(am))
    return e.value, e2.value, am.value


def build_table(lnW: np.ndarray) -> np.ndarray:
    lnW = np.ascontiguousarray(lnW, np.float64)
    T = np.zeros((lnW.size, TCOLS), np.uint32)
    lib().orc_build_table(lnW.size, lnW, T)
    return T


def build_table_mag(L: int, beta: float, lnW: np.ndarray) -> np.ndarray:
    """Multimagnetic thresholds [N+1][10]: row m (up spins), column j + 5u
    (u = 1 for an up spin, flip changes k by 2j - 4 and m by -1 or +1)."""
    lnW = np.ascontiguousarray(lnW, np.float64)
    assert lnW.size == L * L + 1
    T = np.zeros((lnW.size, TCOLS_MAG), np.uint32)
    lib().orc_build_table_mag(L, float(beta), lnW, T)
    return T


def bruteforce_mag(L: int, beta: float):
    """Exact canonical P(m) and the mean bond count k at each m, by
    enumerating all 2^N Ising states (m = number of up spins)."""
    p, km = np.zeros(L * L + 1), np.zeros(L * L + 1)
    lib().orc_bruteforce_mag(L, float(beta), p, km)
    return p, km


def energies(model: int, L: int) -> np.ndarray:
    """E of every bin k: Ising E = -2N + 2k (Eq. 3), Potts E = -2N + k (Eq. 4)."""
    N = L * L
    k = np.arange(2 * N + 1, dtype=np.float64)
    return -2.0 * N + (2.0 * k if model == ISING else k)


# ------------------------------------------------------------------ flatness

@dataclass
class Flatness:
    covered: bool
    flat: bool
    min_over_max: float
    min_over_avg: float
    max_over_avg: float
    k_lo: int
    k_hi: int
    visited: int
    reachable: int


def flatness(H: np.ndarray, mask: np.ndarray, ratio: float = 0.5, rule: int = 0) -> Flatness:
    """Flatness over the reachable bins.  rule 0: every reachable bin visited
    and min/max >= ratio.  rule 1 (the paper's, Sec. 3): every reachable bin
    visited and every entry within [avg/2, 2 avg]."""
    h = H[mask].astype(np.float64)
    nz = np.nonzero(H > 0)[0]
    covered = bool(np.all(h > 0))
    hmax, hmin, havg = float(h.max()), float(h.min()), float(h.mean())
    mom = hmin / hmax if hmax > 0 else 0.0
    if rule == 0:
        flat = covered and mom >= ratio
    else:
        flat = covered and bool(np.all(h >= 0.5 * havg)) and bool(np.all(h <= 2.0 * havg))
    return Flatness(covered, flat, mom, hmin / havg if havg > 0 else 0.0,
                    hmax / havg if havg > 0 else 0.0,
                    int(nz[0]) if nz.size else -1, int(nz[-1]) if nz.size else -1,
                    int(nz.size), int(mask.sum()))


# ------------------------------------------------------------------ run state

class OracleRun:
    """One MUCA problem on the CPU: spins, per-chain state, lnW and T."""

    def __init__(self, model: int, L: int, n_chains: int, seed: int, q: int = 2,
                 n_threads: Optional[int] = None, chain0: int = 0, beta: float = 0.0):
        """Chains chain0 .. chain0 + n_chains - 1 of the problem (a chain's
        trajectory depends only on the seed, its index and lnW).  beta: the
        fixed inverse temperature of the multimagnetic ensemble (ISING_MAG)."""
        self.model, self.L, self.q, self.seed = model, L, q if model == POTTS else 2, seed
        self.beta = float(beta)
        self.N = L * L
        self.n_bins = n_bins_of(model, L)
        self.n_chains = n_chains
        self.chain0 = chain0
        self.n_threads = n_threads or default_threads()
        self.spins = np.zeros((n_chains, self.N), np.uint8)
        self.k = np.zeros(n_chains, np.int32)
        self.m = np.zeros(n_chains, np.int32)
        lib().orc_init(model, self.q, L, chain0, n_chains, seed, self.spins, self.k, self.m)
        self.lnW = np.zeros(self.n_bins, np.float64)
        self.T = self._table()
        self.hist = np.zeros((n_chains, self.n_bins), np.int32)
        self.sabs = np.zeros((n_chains, self.n_bins), np.int64)
        self.sweep = 0
        self.mask = reachable(model, self.q, L)

    def _table(self) -> np.ndarray:
        if self.model == ISING_MAG:
            return build_table_mag(self.L, self.beta, self.lnW)
        return build_table(self.lnW)

    def set_log_weights(self, lnW: np.ndarray):
        self.lnW = np.array(lnW, np.float64)
        self.T = self._table()

    def sweeps(self, n: int, record: int):
        lib().orc_sweeps(self.model, self.q, self.L, self.chain0, self.n_chains, self.seed, self.sweep, n, record,
                         self.T, self.spins, self.k, self.m, self.hist, self.sabs, self.n_threads)
        self.sweep += n

    def merged(self) -> np.ndarray:
        H = np.zeros(self.n_bins, np.int64)
        lib().orc_merge(self.n_chains, self.n_bins, self.hist, H)
        return H

    def iterate(self, n_sweeps: int, ratio: float = 0.5, rule: int = 0, correct: bool = False,
                norm: bool = False):
        """One weight iteration: sweeps with histograms, merge, flatness on
        the merged histogram, recursion (with norm, its update shifted to zero
        mean over the visited bins; optionally followed by the correction
        function), new table, cleared histograms."""
        self.hist[:] = 0
        self.sweeps(n_sweeps, REC_MUCA)
        H = self.merged()
        fl = flatness(H, self.mask, ratio, rule)
        per_chain = self.hist.copy()
        (lib().orc_recursion_norm if norm else lib().orc_recursion)(self.n_bins, H, self.lnW)
        if correct:
            correction(self.lnW, H, self.mask, self.L)
        self.T = self._table()
        self.hist[:] = 0
        return H, fl, per_chain

    def production(self, n_therm: int, n_prod: int):
        self.sweeps(n_therm, REC_NONE)
        self.hist[:] = 0
        self.sabs[:] = 0
        self.sweeps(n_prod, REC_PROD)
        cnt = self.hist.astype(np.int64).sum(axis=0)
        sab = self.sabs.sum(axis=0)
        return cnt, sab


# ------------------------------------------------------------------ correction

def correction(lnW: np.ndarray, H: np.ndarray, mask: np.ndarray, L: int) -> None:
    """The correction function of Sec. 3, in place: outside the sampled
    region [lo, hi] (bins with H > 0) the log-weights continue on the straight
    line through the edge bin and the bin L reachable bins inward (or the far
    edge when the region is narrower)."""
    nz = np.nonzero(H > 0)[0]
    if nz.size == 0:
        return
    lo, hi = int(nz[0]), int(nz[-1])
    if lo == hi:
        return

    def inward(edge, step):
        k, count = edge, 0
        while count < L:
            nk = k + step
            if nk < lo or nk > hi:
                break
            k = nk
            if mask[k]:
                count += 1
        return k

    a, b = inward(lo, 1), inward(hi, -1)
    if a != lo:
        slope = (lnW[lo] - lnW[a]) / float(lo - a)
        for k in range(0, lo):
            if mask[k]:
                lnW[k] = lnW[lo] + slope * float(k - lo)
    if b != hi:
        slope = (lnW[hi] - lnW[b]) / float(hi - b)
        for k in range(hi + 1, lnW.size):
            if mask[k]:
                lnW[k] = lnW[hi] + slope * float(k - hi)


# ------------------------------------------------------------------ reweighting

def reweight(model: int, L: int, lnW: np.ndarray, cnt: np.ndarray, sabs: np.ndarray,
             betas: Sequence[float]):
    """Time-series reweighting, Eq. (2), grouped by energy bin.

    Every measurement in bin k carries weight exp(-beta E_k) / W(E_k); a bin
    with cnt_k measurements and |M| sum S_k contributes cnt_k and S_k times
    that weight.  Returns <E>/N, C_V = beta^2 (<E^2> - <E>^2) / N (the
    specific heat of Sec. 5) and <|M|>/N, all in float64.
    """
    N = L * L
    E = energies(model, L)
    sel = cnt > 0
    Ek, lw = E[sel], np.asarray(lnW, np.float64)[sel]
    ck, sk = cnt[sel].astype(np.float64), sabs[sel].astype(np.float64)
    e_out, c_out, m_out = [], [], []
    for beta in betas:
        a = np.log(ck) - lw - beta * Ek
        A = a.max()
        w = np.exp(a - A)
        Z = w.sum()
        em = (w * Ek).sum() / Z
        var = (w * (Ek - em) ** 2).sum() / Z
        # |M| sums carry the same per-measurement weight exp(-lnW - beta E)
        am = (sk * np.exp(-lw - beta * Ek - A)).sum() / Z
        e_out.append(em / N)
        c_out.append(beta * beta * var / N)
        m_out.append(am / N)
    return np.array(e_out), np.array(c_out), np.array(m_out)


# ------------------------------------------------------------------ interface tension

def _log_canonical(model: int, L: int, lnW: np.ndarray, cnt: np.ndarray, beta: float):
    """Bins with data and their log canonical probability, up to a constant:
    a measurement in bin k carries exp(-beta E_k) / W(E_k) (Eq. 2), so
    ln P_beta(k) = ln cnt_k - lnW_k - beta E_k."""
    E = energies(model, L)
    ks = np.flatnonzero(np.asarray(cnt) > 0)
    a = np.log(np.asarray(cnt, np.float64)[ks]) - np.asarray(lnW, np.float64)[ks] - beta * E[ks]
    return ks, a


def _best_valley(a: np.ndarray):
    """Score of each point as the bottom of a double peak: its depth below the
    lower of the highest values on its two sides (itself included), less
    |ln(M_left / M_right)|, M the probability (sum of e^a) on each side, the
    point included in both.  The two phases of a double peak carry comparable
    probability; an isolated bin at an edge or a dip in a tail does not, and
    scores below zero.  Returns the first best point and its score."""
    left = np.maximum.accumulate(a)
    right = np.maximum.accumulate(a[::-1])[::-1]
    w = np.exp(a - a.max())
    m_left = np.cumsum(w)
    m_right = np.cumsum(w[::-1])[::-1]
    with np.errstate(divide="ignore"):   # a side whose e^a underflows scores -inf
        score = np.minimum(left, right) - a - np.abs(np.log(m_left) - np.log(m_right))
    i = int(np.argmax(score))
    return i, float(score[i])


def _valley_split(model, L, lnW, cnt, beta_lo, beta_hi):
    """The bin that separates the ordered from the disordered peak.

    Reading: the two peaks are separated at the valley of the reweighted
    histogram, taken where the histogram is most clearly double-peaked: over 65
    equally spaced beta in the bracket, the best-scoring valley (its depth less
    the log ratio of the probabilities on its two sides) at the beta where
    that score is highest.  A split fixed in k makes the peak-height
    difference below a continuous, increasing function of beta."""
    best, split = 0.0, None
    for i in range(65):
        b = beta_lo + (beta_hi - beta_lo) * i / 64.0
        ks, a = _log_canonical(model, L, lnW, cnt, b)
        j, score = _best_valley(a)
        if score > best:
            best, split = score, int(ks[j])
    if split is None:
        raise ValueError("no two peaks")
    return split


def _two_peaks(model, L, lnW, cnt, beta, split):
    """The ordered and disordered peaks (the largest ln P at k <= split and at
    k > split) and the smallest ln P between them."""
    ks, a = _log_canonical(model, L, lnW, cnt, beta)
    low, high = ks <= split, ks > split
    if not low.any() or not high.any():
        raise ValueError("no two peaks")
    i_o = np.flatnonzero(low)[np.argmax(a[low])]
    i_d = np.flatnonzero(high)[np.argmax(a[high])]
    i_m = i_o + int(np.argmin(a[i_o:i_d + 1]))
    return (int(ks[i_o]), int(ks[i_m]), int(ks[i_d])), (a[i_o], a[i_m], a[i_d])


def interface_tension(model: int, L: int, lnW, cnt, beta_lo: float, beta_hi: float):
    """Order-disorder interface tension, Eq. (9), Sec. 5.

    Step 1: find the inverse temperature at which the histogram reweighted to
    the canonical ensemble has its two peaks at the same height (bisection on
    the difference of the two log peak heights on either side of the valley
    bin, which grows with beta because the ordered side has the lower
    energies).  Step 2: sigma_od = ln(P_max/P_min) / (2L) there, with P_max
    the common peak height.  Returns (beta, sigma, (k_ordered, k_min,
    k_disordered))."""
    lo, hi = float(beta_lo), float(beta_hi)
    split = _valley_split(model, L, lnW, cnt, lo, hi)

    def gap(beta):
        _, (ao, _, ad) = _two_peaks(model, L, lnW, cnt, beta, split)
        return ao - ad
    if not (gap(lo) < 0.0 < gap(hi)):
        raise ValueError("peak heights do not cross in the bracket")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if not (lo < mid < hi):
            break
        if gap(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    ks, (ao, am, ad) = _two_peaks(model, L, lnW, cnt, beta, split)
    if not ks[0] < ks[1] < ks[2]:
        raise ValueError("no minimum between the peaks: one peak only")
    return beta, (0.5 * (ao + ad) - am) / (2.0 * L), ks
