"""Exact results for the finite 2D periodic Ising model (test pins only).

Kaufman (1949) gives the partition function of the L x L torus as a sum of
four products over the lattice's Onsager angles; Beale (1996) observed that,
read as a polynomial in x = exp(-2K), it yields the exact density of states.
This module evaluates that polynomial at complex roots of unity with mpmath
and inverts the discrete Fourier transform to get Omega(k) for every number k
of unsatisfied bonds.  Everything here is independent of the oracle and of
the product library: it is a closed form, not a sampler.

With K = beta J and E = -2N + 2k, the partition function is
    Z = sum_k Omega_k exp(2NK) x^k,   so   P(x) = sum_k Omega_k x^k = Z x^N.
Kaufman:  Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4), with
    cosh g_l = cosh 2K coth 2K - cos(pi l / L),
    Z1 = prod_{l odd} 2 cosh(L g_l / 2),   Z2 = prod_{l odd} 2 sinh(L g_l / 2),
    Z3 = prod_{l even} 2 cosh(L g_l / 2),  Z4 = prod_{l even} 2 sinh(L g_l / 2),
for l in 0..2L-1, where g_0 = 2K + ln tanh K carries its sign.  Pairing l with
2L - l turns each pair into 2 + 2 T_L(c_l) or 2 T_L(c_l) - 2 (T_L the
Chebyshev polynomial), which is rational in x and free of square roots.
"""
import functools

import mpmath
import numpy as np


def _cheb(L: int, c):
    """Chebyshev T_L(c) by the three-term recurrence."""
    t0, t1 = mpmath.mpf(1), c
    if L == 0:
        return t0
    for _ in range(L - 1):
        t0, t1 = t1, 2 * c * t1 - t0
    return t1


def poly_value(L: int, x):
    """P(x) = sum_k Omega_k x^k for the L x L torus (L even), at complex x."""
    assert L % 2 == 0 and L >= 2
    N = L * L
    one = mpmath.mpf(1)
    base = (one + x * x) ** 2 / (2 * x * (one - x * x))
    z1 = z2 = z3 = z4 = mpmath.mpc(1)
    for l in range(1, L, 2):
        t = _cheb(L, base - mpmath.cos(mpmath.pi * l / L))
        z1 *= 2 + 2 * t
        z2 *= 2 * t - 2
    for l in range(2, L, 2):
        t = _cheb(L, base - mpmath.cos(mpmath.pi * l / L))
        z3 *= 2 + 2 * t
        z4 *= 2 * t - 2
    g0 = (one - x) / (x * (one + x))   # exp(g_0), g_0 = 2K + ln tanh K
    gL = (one + x) / (x * (one - x))   # exp(g_L)
    h = L // 2
    z3 *= (g0 ** h + g0 ** (-h)) * (gL ** h + gL ** (-h))
    z4 *= (g0 ** h - g0 ** (-h)) * (gL ** h - gL ** (-h))
    pref = ((one - x * x) / x) ** (N // 2) / 2
    return x ** N * pref * (z1 + z2 + z3 + z4)


@functools.lru_cache(maxsize=None)
def density_of_states(L: int) -> tuple:
    """Exact Omega(k), k = 0..2N, as Python ints (L even)."""
    N = L * L
    J = 2 * N + 1
    with mpmath.workdps(int((N + 192) * 0.30103) + 10):
        xs = [mpmath.exp(2j * mpmath.pi * (j + mpmath.mpf(1) / 4) / J) for j in range(J)]
        ps = [poly_value(L, x) for x in xs]
        omega = []
        for k in range(J):
            acc = mpmath.mpc(0)
            for j in range(J):
                acc += ps[j] * xs[j] ** (-k)
            v = acc / J
            omega.append(int(mpmath.nint(v.real)))
    return tuple(omega)


def log_dos(L: int) -> np.ndarray:
    """ln Omega(k) as float64 (-inf where Omega = 0)."""
    om = density_of_states(L)
    out = np.full(len(om), -np.inf)
    for k, v in enumerate(om):
        if v > 0:
            out[k] = float(mpmath.log(v))
    return out


def kaufman_lnZ(L: int, K):
    """ln Z of the L x L torus at coupling K = beta J, straight from Kaufman's
    four products (no density of states involved)."""
    K = mpmath.mpf(K)
    N = L * L
    cc = mpmath.cosh(2 * K) / mpmath.tanh(2 * K)
    gam = []
    for l in range(2 * L):
        if l == 0:
            gam.append(2 * K + mpmath.log(mpmath.tanh(K)))
        else:
            gam.append(mpmath.acosh(cc - mpmath.cos(mpmath.pi * l / L)))
    z1 = z2 = z3 = z4 = mpmath.mpf(1)
    for l in range(2 * L):
        a = L * gam[l] / 2
        if l % 2:
            z1 *= 2 * mpmath.cosh(a)
            z2 *= 2 * mpmath.sinh(a)
        else:
            z3 *= 2 * mpmath.cosh(a)
            z4 *= 2 * mpmath.sinh(a)
    return mpmath.log((2 * mpmath.sinh(2 * K)) ** (mpmath.mpf(N) / 2) / 2 * (z1 + z2 + z3 + z4))


def kaufman_energy_cv(L: int, beta: float):
    """<E>/N and C_V = beta^2 var(E)/N from derivatives of Kaufman's ln Z."""
    N = L * L
    with mpmath.workdps(40):
        f = lambda b: kaufman_lnZ(L, b)
        d1 = mpmath.diff(f, beta, 1)
        d2 = mpmath.diff(f, beta, 2)
        return float(-d1 / N), float(beta * beta * d2 / N)
