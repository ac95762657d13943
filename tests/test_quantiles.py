"""Interval quantiles in the library's host code (no GPU): the standard
normal quantile (credible level of the Bayesian-cubature interval) and the
Student-t quantile (the RQMC interval, eq. RQMC).

Pinned by closed forms (the Cauchy quantile for one degree of freedom, the
two-degree form, textbook normal values) and by the residual of an
independent distribution function: scipy's tail functions evaluated at the
library's quantile must give back the requested tail probability."""
import math

import numpy as np
import pytest
from scipy import special, stats

import paper_2502_14256_amd as ldk


def test_normal_textbook_values():
    # z_{0.975} and z_{0.995} to 16 digits (standard tables)
    assert abs(ldk.normal_quantile(0.975) - 1.959963984540054) < 4e-16 * 1.96
    assert abs(ldk.normal_quantile(0.995) - 2.5758293035489004) < 4e-16 * 2.58
    assert ldk.normal_quantile(0.5) == 0.0
    # odd symmetry, up to the rounding of 1 - p (|dx| = |dp| / phi(x))
    for p in (1e-9, 0.01, 0.2, 0.45):
        x = ldk.normal_quantile(p)
        phi = math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)
        assert abs(x + ldk.normal_quantile(1.0 - p)) <= 2e-16 / phi + 8e-16 * abs(x)


@pytest.mark.parametrize("p", list(np.logspace(-300, -1, 60)) + list(np.linspace(0.02, 0.98, 49)))
def test_normal_residual(p):
    x = ldk.normal_quantile(p)
    # the tail probability at x, from the smaller tail (erfc), matches p
    got = special.ndtr(x) if p < 0.5 else special.ndtr(-x)
    want = p if p < 0.5 else 1.0 - p
    # |dPhi| = phi(x) |dx|: a quantile good to 4 ulps moves the tail by
    # 4 u |x| phi(x) relative to it, plus the tail function's own rounding
    phi = math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)
    tol = 4e-16 * abs(x) * phi + 4e-16 * want
    assert abs(got - want) <= tol, (p, x, got, want)


def test_student_t_closed_forms():
    for p in (1e-12, 1e-6, 0.01, 0.1, 0.3, 0.7, 0.9, 0.975, 0.995, 1 - 1e-9):
        # one degree of freedom: the Cauchy quantile tan(pi (p - 1/2)),
        # exact in extended precision here
        want1 = float(math.tan(math.pi * (p - 0.5))) if 1e-3 < p < 1 - 1e-3 else \
            (-1.0 / math.tan(math.pi * p) if p < 0.5 else 1.0 / math.tan(math.pi * (1 - p)))
        assert abs(ldk.student_t_quantile(p, 1) - want1) <= 1e-13 * abs(want1)
        # two degrees of freedom: (2p - 1) / sqrt(2 p (1 - p))
        want2 = (2 * p - 1) / math.sqrt(2 * p * (1 - p))
        assert abs(ldk.student_t_quantile(p, 2) - want2) <= 1e-14 * abs(want2)
    # large dof tends to the normal quantile: |t - z| = O(1/dof)
    z = ldk.normal_quantile(0.995)
    assert abs(ldk.student_t_quantile(0.995, 65534) - z) < 1e-4


@pytest.mark.parametrize("dof", [3, 4, 5, 9, 15, 63, 64, 255, 1000, 65534])
def test_student_t_residual(dof):
    for p in [1e-9, 1e-3, 0.005, 0.025, 0.1, 0.3, 0.6, 0.9, 0.95, 0.975, 0.99, 0.995, 0.9995]:
        t = ldk.student_t_quantile(p, dof)
        # independent distribution function (scipy's stdtr, from the
        # incomplete beta function of cephes)
        tail = special.stdtr(dof, -abs(t))
        want = p if p < 0.5 else 1.0 - p
        dens = stats.t.pdf(t, dof)
        # quantile good to ~1e-13 relative (the incomplete beta's prefactor
        # loses digits to lgamma at large dof), plus the reference's rounding
        tol = 1e-13 * abs(t) * dens * (1 + dof / 1000.0) + 1e-14 * want
        assert abs(tail - want) <= tol, (dof, p, t, tail, want)
        assert (t < 0) == (p < 0.5)


def test_student_t_agrees_with_scipy_ppf():
    # scipy's ppf itself carries ~1e-11 relative error (see the residual
    # tests), so agreement is only checked to 1e-9
    for dof in (3, 9, 30, 1000):
        for p in (0.95, 0.975, 0.995):
            a, b = ldk.student_t_quantile(p, dof), stats.t.ppf(p, dof)
            assert abs(a - b) <= 1e-9 * abs(b)


def test_quantile_argument_errors():
    assert math.isnan(ldk.lib().ldk_normal_quantile(0.0))
    assert math.isnan(ldk.lib().ldk_normal_quantile(1.0))
    with pytest.raises(ldk.LdkError):
        ldk.student_t_quantile(0.5, 0)
    with pytest.raises(ldk.LdkError):
        ldk.normal_quantile(1.5)
