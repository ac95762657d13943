"""Pins for the oracle's kernel factors (Sec. 5.2, Sec. 5.3, Theorem 1), CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from golden_io import frac, rows


def _delta(x: Fraction) -> int:
    v = x * 2**64
    assert v.denominator == 1
    return int(v)


def test_walsh_convention_matches_lemma():
    # Lemma of Appendix B: fixes wal_{2^a}(x) = (-1)^{xi_{a+1}}
    for p, k, v in rows("walsh_monomial_coefficients.txt"):
        assert brute.walsh_coefficient_monomial(int(p), int(k)) == frac(v), (p, k)


def test_s4tilde_zero_is_printed_value():
    # proof of Theorem 1: s~_4(0) = 1/294
    assert abs(brute.dsi_series_s4_at_zero() - Fraction(1, 294)) < Fraction(1, 10**40)


@pytest.mark.parametrize("alpha", [2, 3, 4])
def test_series_organisation_equals_literal_partial_sum(alpha):
    rng = np.random.default_rng(alpha)
    for _ in range(6):
        delta = int(rng.integers(0, 2**10)) << 54
        assert brute.dsi_series(alpha, delta, A=10) == brute.dsi_series_literal(
            alpha, delta, 2**10)


def test_special_values_theorem1(orc):
    for a, x, v in rows("dsi_special_values.txt"):
        if a == "s4tilde":
            continue
        delta = _delta(frac(x))
        assert abs(orc.dsi_factor(int(a), delta) - float(frac(v))) < 1e-15
        assert abs(brute.dsi_series(int(a), delta) - frac(v)) < Fraction(1, 10**40)


@pytest.mark.parametrize("alpha", [2, 3, 4])
def test_dsi_closed_form_matches_series(orc, alpha):
    rng = np.random.default_rng(100 + alpha)
    deltas = [0, 1, 2**63, 2**62 + 1, (1 << 64) - 1]
    deltas += [int(v) for v in rng.integers(0, 2**64, size=20, dtype=np.uint64)]
    # short and deep digit strings (large beta)
    deltas += [int(v) >> int(s) for v, s in zip(rng.integers(0, 2**64, size=20, dtype=np.uint64),
                                                 rng.integers(1, 60, size=20))]
    for delta in deltas:
        series = float(brute.dsi_series(alpha, delta))
        assert abs(orc.dsi_factor(alpha, delta) - series) < 4e-15, (alpha, delta)


def test_dsi_order1_reading_matches_its_series(orc):
    # alpha = 1 is a reading (K_1 = 1 - 3 t_1): parity unpinned against the
    # paper; this only checks the closed form against its own Walsh series.
    rng = np.random.default_rng(7)
    deltas = [0, 2**63, 2**62, 3 << 62, 5 << 60]
    deltas += [int(v) for v in rng.integers(0, 2**64, size=30, dtype=np.uint64)]
    for delta in deltas:
        assert abs(orc.dsi_factor(1, delta) - float(brute.dsi1_series(delta))) < 1e-15
    assert orc.dsi_factor(1, 0) == 1.0
    assert orc.dsi_factor(1, 2**63) == -0.5
    assert orc.dsi_factor(1, 2**62) == 0.25
    # literal partial sum of the reading's series over k < 2^L
    for delta in (0, 5 << 60, 13 << 58):
        lit = sum((Fraction(brute.walsh(k, delta), 2 ** (2 * (k.bit_length() - 1) + 1))
                   for k in range(1, 2**8)), Fraction(0))
        assert lit == brute.dsi1_series(delta, A=8)


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_si_factor_matches_fourier_series(orc, alpha):
    rng = np.random.default_rng(alpha)
    deltas = [0, 2**63, 2**62, 3 << 62] + [int(v) for v in
                                           rng.integers(0, 2**64, size=12, dtype=np.uint64)]
    for delta in deltas:
        x = float(delta) * 2.0**-64
        s, tail = brute.si_series(alpha, x)
        assert abs(orc.si_factor(alpha, delta) - s) <= tail + 1e-12 * (1 + abs(s))


def test_si_special_values(orc):
    pi = math.pi
    assert abs(orc.si_factor(1, 0) - pi**2 / 3) < 1e-13
    assert abs(orc.si_factor(1, 2**63) + pi**2 / 6) < 1e-13
    assert abs(orc.si_factor(2, 0) - pi**4 / 45) < 1e-12
    assert abs(orc.si_factor(2, 2**63) + 7 * pi**4 / 360) < 1e-12
    assert abs(orc.si_factor(3, 0) - 2 * pi**6 / 945) < 1e-11
