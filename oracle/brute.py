"""Brute-force layer of the oracle (TEST INFRASTRUCTURE ONLY).

Independent routes to the quantities the C oracle computes, used by the
``not gpu`` tests to pin it.  Everything here is written from the paper's
definitions, in exact rationals where the quantity is rational:

* Walsh functions (Sec. 5.3): for k = sum_l 2^{a_l},
  wal_k(x) = prod_l (-1)^{xi_{a_l + 1}}, xi_t the t-th binary digit of x.
* The DSI kernel series, eq. (DSI_kernel):
  K_alpha(x) = sum_{k >= 1} wal_k(x) / 2^{mu_alpha(k)},
  mu_alpha(k) = sum_{l <= min(alpha, #k)} (a_l + 1).
* Walsh coefficients of x^p (Lemma of Appendix B), by exact integration over
  dyadic intervals.
* The SI kernel's Fourier series (Sec. 5.2):
  K_alpha(x) = sum_{h != 0} exp(2 pi i h x) / |h|^{2 alpha}.
* Eigenvalues of d = 1 Gram matrices by aliasing sums of the Walsh / Fourier
  coefficients.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def digits(delta: int, count: int) -> list[int]:
    """Binary digits xi_1..xi_count of x = delta * 2^-64 (zero past the 64th)."""
    return [((delta >> (64 - t)) & 1) if t <= 64 else 0 for t in range(1, count + 1)]


def frac_value(delta: int) -> Fraction:
    return Fraction(delta, 2**64)


def walsh(k: int, delta: int) -> int:
    """wal_k(x) for x = delta * 2^-64 (base 2, Sec. 5.3)."""
    s, a = 0, 0
    while k >> a:
        if (k >> a) & 1:
            s ^= ((delta >> (63 - a)) & 1) if a < 64 else 0
        a += 1
    return -1 if s else 1


def _mu(alpha: int, k: int) -> int:
    bits = [a for a in range(k.bit_length() - 1, -1, -1) if (k >> a) & 1]
    return sum(a + 1 for a in bits[:alpha])


def dsi_series(alpha: int, delta: int, A: int = 200) -> Fraction:
    """Exact-rational evaluation of eq. (DSI_kernel), alpha >= 2.

    Organised by the positions of the leading bits of k, as in the proof of
    Theorem 1: terms with #k = nu < alpha contribute prod_l w_{a_l} with
    w_a = wal_{2^a}(x) 2^{-(a+1)}; terms with #k >= alpha are summed over the
    free lower part k' < 2^{a_alpha} using
    sum_{k' < 2^a} wal_{k'}(x) = prod_{t < a} (1 + wal_{2^t}(x)),
    which follows from wal being multiplicative over the bits of k.
    Bit positions a >= A are dropped (their total is below 2^-A A^alpha).
    """
    if alpha < 2:
        raise ValueError("the series defines K_alpha for alpha >= 2")
    xi = digits(delta, A)
    w = [Fraction(-1 if xi[a] else 1, 2 ** (a + 1)) for a in range(A)]
    # P[a] = sum_{k' < 2^a} wal_k'(x)
    P = [Fraction(1)]
    for a in range(A):
        P.append(P[-1] * (1 + (-1 if xi[a] else 1)))
    # E[a][nu] = e_nu(w_a, ..., w_{A-1}) (elementary symmetric polynomials)
    E = [[Fraction(0)] * (alpha + 1) for _ in range(A + 1)]
    E[A][0] = Fraction(1)
    for a in range(A - 1, -1, -1):
        for nu in range(alpha + 1):
            E[a][nu] = E[a + 1][nu] + (w[a] * E[a + 1][nu - 1] if nu > 0 else 0)
    total = sum((E[0][nu] for nu in range(1, alpha)), Fraction(0))
    # #k >= alpha: choose a_alpha = a, then alpha-1 larger positions
    for a in range(A):
        if P[a] == 0:
            continue
        total += w[a] * P[a] * E[a + 1][alpha - 1]
    return total


def dsi_series_s4_at_zero(A: int = 200) -> Fraction:
    """s~_4(0) of Appendix B: sum over #k >= 4 at x = 0."""
    w = [Fraction(1, 2 ** (a + 1)) for a in range(A)]
    E = [[Fraction(0)] * 4 for _ in range(A + 1)]
    E[A][0] = Fraction(1)
    for a in range(A - 1, -1, -1):
        for nu in range(4):
            E[a][nu] = E[a + 1][nu] + (w[a] * E[a + 1][nu - 1] if nu > 0 else 0)
    return sum((w[a] * 2**a * E[a + 1][3] for a in range(A)), Fraction(0))


def dsi1_series(delta: int, A: int = 200) -> Fraction:
    """Walsh series of the order-1 reading: Walsh coefficient 2^{-2 a_1 - 1}
    for k >= 1 (a_1 = leading bit of k), summed over k' < 2^{a_1} as above."""
    xi = digits(delta, A)
    total = Fraction(0)
    Pa = Fraction(1)
    for a in range(A):
        wal_top = -1 if xi[a] else 1
        total += Fraction(wal_top, 2 ** (2 * a + 1)) * Pa
        Pa *= 1 + wal_top
    return total


def dsi_series_literal(alpha: int, delta: int, kmax: int) -> Fraction:
    """The literal partial sum over 1 <= k < kmax of eq. (DSI_kernel)."""
    return sum((Fraction(walsh(k, delta), 2 ** _mu(alpha, k)) for k in range(1, kmax)),
               Fraction(0))


def walsh_coefficient_monomial(p: int, k: int) -> Fraction:
    """int_0^1 x^p wal_k(x) dx exactly: wal_k is constant on dyadic intervals
    of length 2^-L, L = bit length of k."""
    L = max(k.bit_length(), 1)
    total = Fraction(0)
    for j in range(2**L):
        delta = j << (64 - L)
        lo, hi = Fraction(j, 2**L), Fraction(j + 1, 2**L)
        total += walsh(k, delta) * (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)
    return total


def si_series(alpha: int, x: float, H: int = 200000) -> tuple[float, float]:
    """Truncated Fourier series 2 sum_{h=1}^{H} cos(2 pi h x) / h^{2 alpha}
    and its tail bound 2 / ((2 alpha - 1) H^{2 alpha - 1})."""
    h = np.arange(1, H + 1, dtype=np.float64)
    s = 2.0 * np.sum(np.cos(2.0 * math.pi * h * x) / h ** (2 * alpha))
    return float(s), 2.0 / ((2 * alpha - 1) * H ** (2 * alpha - 1))


def net_alias_sum(alpha: int, k: int, m: int, B: int = 72) -> Fraction:
    """sum over h >= 0 with h == k (mod 2^m) of r(h), r(0) = 1,
    r(h) = 2^{-mu_alpha(h)} (Walsh coefficients of 1 + K_alpha).

    Terms are grouped by the leading bit b + m of h (b >= 0); the free bits
    between it and the fixed low m bits are enumerated by a digit recursion
    that tracks how many leading ones have been seen (only the first alpha
    count in mu_alpha).  Groups with b >= B are dropped."""
    total = Fraction(1) if k == 0 else Fraction(1, 2 ** _mu(alpha, k))
    for b in range(B):
        top = b + m
        # state: number of set bits seen (capped at alpha) -> accumulated weight
        state = {1: Fraction(1, 2 ** (top + 1))} if alpha >= 1 else {0: Fraction(1)}
        for p in range(top - 1, -1, -1):
            new: dict[int, Fraction] = {}
            choices = (0, 1) if p >= m else (((k >> p) & 1),)
            for cnt, wgt in state.items():
                for bit in choices:
                    if bit:
                        c2 = min(cnt + 1, alpha + 1)
                        w2 = wgt * (Fraction(1, 2 ** (p + 1)) if cnt < alpha else 1)
                    else:
                        c2, w2 = cnt, wgt
                    new[c2] = new.get(c2, Fraction(0)) + w2
            state = new
        total += sum(state.values(), Fraction(0))
    return total


def lattice_alias_sum(alpha: int, k: int, n: int) -> float:
    """sum over h == k (mod n) of c(h), c(0) = 1, c(h) = |h|^{-2 alpha}
    (Fourier coefficients of 1 + K_alpha), via Hurwitz zeta sums."""
    from scipy.special import zeta

    s = 2 * alpha
    if k % n == 0:
        return 1.0 + 2.0 * float(zeta(s, 1.0)) / n**s
    q = (k % n) / n
    return (float(zeta(s, q)) + float(zeta(s, 1.0 - q))) / n**s


def hadamard(m: int) -> np.ndarray:
    """Unnormalised Hadamard matrix H_m, H_{k j} = (-1)^{popcount(k & j)}."""
    n = 2**m
    idx = np.arange(n)
    pc = np.vectorize(lambda v: bin(int(v)).count("1"))(idx[:, None] & idx[None, :])
    return np.where(pc % 2 == 0, 1.0, -1.0)


def bitrev(j: int, m: int) -> int:
    """R_m(j): reverse the m low bits of j."""
    r = 0
    for t in range(m):
        r |= ((j >> t) & 1) << (m - 1 - t)
    return r


def fourier_br(m: int) -> np.ndarray:
    """conj(T_m) = {W_m^{k R_m(j)}} of Sec. 5.2 (unnormalised)."""
    n = 2**m
    R = np.array([bitrev(j, m) for j in range(n)])
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, R) / n)
