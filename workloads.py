"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only names problem shapes, seeds and run lengths.  It holds no
arithmetic of the method: every random number a run draws comes from the
counter-based generator keyed by the seeds named here, which the product
library and the oracle each implement on their own.

The paper runs no dataset: its inputs are lattices started at infinite
temperature (random spins) from a seed (Sec. 3, "Systems and Implementation
Issues").  The shapes below are the workloads the paper studies (2D periodic
Ising and 8-state Potts, Sec. 3) at the sizes of the measured configurations.
"""
import math
from dataclasses import dataclass, field
from typing import List, Tuple

ISING = 0
POTTS = 1
ISING_MAG = 2   # Ising with multimagnetic weights over M at a fixed beta (Sec. 4)


@dataclass(frozen=True)
class Problem:
    """One MUCA problem: a model, a lattice size and a set of chains."""
    model: int          # ISING or POTTS
    L: int              # linear lattice size, N = L*L sites, periodic
    n_chains: int       # independent Markov chains sharing lnW
    seed: int           # 64-bit key of the counter-based generator
    q: int = 2          # number of Potts states (2 for Ising)
    beta: float = 0.0   # fixed inverse temperature of the multimagnetic ensemble

    @property
    def N(self) -> int:
        return self.L * self.L

    @property
    def n_bins(self) -> int:
        # bins are indexed by the number of unsatisfied bonds, 0..2N, or for
        # the multimagnetic ensemble by the number of up spins, 0..N
        return self.N + 1 if self.model == ISING_MAG else 2 * self.N + 1


@dataclass(frozen=True)
class RunPlan:
    problems: Tuple[Problem, ...]
    sweeps_per_iter: int
    n_iters: int
    n_therm: int = 0
    n_prod: int = 0
    betas: Tuple[float, ...] = field(default_factory=tuple)


def beta_grid(n: int = 200, lo: float = 0.3, hi: float = 0.6) -> Tuple[float, ...]:
    """Inverse temperatures for reweighting, endpoints included."""
    return tuple(lo + (hi - lo) * j / (n - 1) for j in range(n))


# Ising L=8, 4 chains, 20 iterations of 1e4 sweeps: small enough for the oracle.
C1 = RunPlan(problems=(Problem(ISING, 8, 4, 1),), sweeps_per_iter=10_000, n_iters=20)

# Ising L=64, 4096 chains, 30 iterations of 2e3 sweeps, then 1e5 production
# sweeps reweighted to 200 inverse temperatures in [0.3, 0.6].
C2 = RunPlan(problems=(Problem(ISING, 64, 4096, 1),), sweeps_per_iter=2_000, n_iters=30,
             n_therm=2_000, n_prod=100_000, betas=beta_grid())

# 8-state Potts L=32, 4096 chains, 50 iterations of 5e3 sweeps.
C3 = RunPlan(problems=(Problem(POTTS, 32, 4096, 1, q=8),), sweeps_per_iter=5_000, n_iters=50)

# Mixed batch in one launch: Ising L in {16,24,32,48,64}, 8-Potts L in {8,16,24,32},
# 512 chains each, seeds 1..9.
_C4_SHAPES = [(ISING, 16), (ISING, 24), (ISING, 32), (ISING, 48), (ISING, 64),
              (POTTS, 8), (POTTS, 16), (POTTS, 24), (POTTS, 32)]
C4 = RunPlan(problems=tuple(Problem(m, L, 512, s + 1, q=(2 if m == ISING else 8))
                            for s, (m, L) in enumerate(_C4_SHAPES)),
             sweeps_per_iter=2_000, n_iters=10)

# Multimagnetic Ising (Sec. 4): weights over the magnetization at beta = (3/2) beta_0,
# L=32 (the largest size of the paper's multimagnetic runs), 4096 chains, 2e3 sweeps.
BETA0_ISING = 0.5 * math.log(1.0 + math.sqrt(2.0))
C_MAG = RunPlan(problems=(Problem(ISING_MAG, 32, 4096, 1, beta=1.5 * BETA0_ISING),), sweeps_per_iter=2_000,
                n_iters=30)

# Learned initial weights: training sizes and seeded test runs.
C5_TRAIN: List[Tuple[int, int]] = [(ISING, 8), (ISING, 16), (ISING, 24), (ISING, 32), (ISING, 48),
                                   (POTTS, 8), (POTTS, 16), (POTTS, 24)]
C5_TEST: List[Tuple[int, int]] = [(ISING, 96), (ISING, 128), (POTTS, 48)]
C5_TEST_CHAINS = 8192
C5_SEEDS = (1, 2, 3)


def small_problem(model: int, L: int, n_chains: int, seed: int) -> Problem:
    return Problem(model, L, n_chains, seed, q=(2 if model == ISING else 8))
