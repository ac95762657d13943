"""Pins for the oracle's RQMC estimate and Student-t interval (eq. RQMC) and
its Genz test integrands: the corner peak against its exact integral and the
paper's printed example, the Koksma-Hlawka bound in one dimension, exactness
of the g = 1 lattice on trigonometric integrands, and the interval against
scipy's.  CPU only."""
import itertools
import math
import statistics

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W
from golden_io import rows


def corner_peak_exact(c):
    """int over [0,1]^d of (1 + c.x)^-(d+1): with
    (1 + s)^-(d+1) = (1/d!) int_0^inf t^d e^{-t(1+s)} dt the integral is
    (1/d!) int_0^inf t^d e^{-t} prod_j (1 - e^{-c_j t}) / (c_j t) dt."""
    d = len(c)

    def g(t):
        if t <= 0.0:
            return 0.0
        lg = d * math.log(t) - t - math.lgamma(d + 1)
        lg += sum(math.log(-math.expm1(-cj * t) / (cj * t)) for cj in c)
        return math.exp(lg)

    val, err = integrate.quad(g, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=500)
    assert err < 1e-12 * val
    return val


def corner_peak_inclusion_exclusion(c):
    """The same integral by inclusion-exclusion over the 2^d vertices:
    (1 / (d! prod c)) sum_S (-1)^|S| / (1 + sum_{j in S} c_j)."""
    d = len(c)
    tot = 0.0
    for S in itertools.product([0, 1], repeat=d):
        tot += (-1) ** sum(S) / (1.0 + sum(cj for cj, s in zip(c, S) if s))
    return tot / (math.factorial(d) * float(np.prod(c)))


@pytest.mark.parametrize("d", [1, 2, 3, 4, 6])
def test_exact_corner_peak_two_ways(d):
    c = np.random.default_rng(d).uniform(0.2, 1.5, d)
    assert abs(corner_peak_exact(c) - corner_peak_inclusion_exclusion(c)) <= 1e-13


def test_paper_example_within_printed_interval():
    # Sec. 6 listing: the exact integral of the d = 50 corner peak lies in the
    # printed 99 % interval muhat +- half_width
    g = {k: float(v) for k, v in rows("rqmc_corner_peak_d50.txt")}
    mu = corner_peak_exact(W.corner_peak_coefficients(int(g["d"])))
    assert abs(mu - g["muhat"]) <= g["half_width"]


def test_oracle_corner_peak_converges_to_exact(orc):
    # the oracle's integrand and RQMC mean on the paper's shape (d = 50,
    # n = 2^15, R = 10; an order-3 interlaced LMS + shifted net)
    d, m, R, alpha = 50, 15, 10, 3
    src = W.small_net(2502, m=m, d=alpha * d, R=R)
    shift = np.random.default_rng(7).integers(0, 2**64, size=(R, d), dtype=np.uint64)
    pts = orc.higher_order_dnet_points(src["gen"], src["lms"], shift, alpha, m, 0, 2**m)
    c = W.corner_peak_coefficients(d)
    est = orc.rqmc(orc.genz_corner_peak(orc.unit_points(pts), c), tau=0.01)
    mu = corner_peak_exact(c)
    assert abs(est["mean"] - mu) <= max(est["half"], 2e-7)
    assert est["half"] < 5e-6


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [3, 6, 9])
def test_koksma_hlawka_d1(orc, kind, m):
    # d = 1 and one point in each [k/n, (k+1)/n): star discrepancy <= 1/n, so
    # |mu_r - mu| <= V(f) / n with V = f(0) - f(1) for the decreasing corner peak
    n, R = 2**m, 4
    shift = np.random.default_rng(m).integers(0, 2**64, size=(R, 1), dtype=np.uint64)
    if kind == "lattice":
        pts = orc.lattice_points(np.array([1], np.uint64), shift, m, 0, n)
    else:
        C = np.array([[np.uint64(1) << np.uint64(63 - k) for k in range(m)]], np.uint64)
        pts = orc.dnet_points(C, None, shift, m, 0, n, R=R)
    for cc in (0.3, 1.0, 4.0):
        est = orc.rqmc(orc.genz_corner_peak(orc.unit_points(pts), [cc]))
        mu = (1.0 - 1.0 / (1.0 + cc)) / cc
        V = 1.0 - (1.0 + cc) ** -2
        assert np.all(np.abs(est["mu_r"] - mu) <= V / n * (1 + 1e-12))


@pytest.mark.parametrize("q", [1, 3, 7, 8, 16])
def test_lattice_integrates_trigonometric_exactly(orc, q):
    # g = 1, n = 8, shift delta: (1/n) sum_k cos(2 pi u + 2 pi q (k/n + delta))
    # is 0 unless n | q, then cos(2 pi u + 2 pi q delta)
    m, n, u = 3, 8, 0.17
    shift = np.array([[np.uint64(0x9E3779B97F4A7C15)]], np.uint64)
    pts = orc.lattice_points(np.array([1], np.uint64), shift, m, 0, n)
    x = orc.unit_points(pts)
    est = orc.rqmc(orc.genz_oscillatory(x, [2 * math.pi * q], u))
    delta = float(shift[0, 0]) * 2.0**-64
    want = math.cos(2 * math.pi * (u + q * delta)) if q % n == 0 else 0.0
    assert abs(est["mu_r"][0] - want) <= 1e-13


def test_interval_against_scipy_and_statistics(orc):
    rng = np.random.default_rng(3)
    for R in (2, 5, 10, 16):
        y = rng.standard_normal((R, 64)) + 2.0
        tau = 0.05
        est = orc.rqmc(y, tau=tau)
        lo, hi = stats.t.interval(1 - tau, R - 1, loc=est["mean"],
                                  scale=est["std"] / math.sqrt(R))
        assert abs((est["mean"] - est["half"]) - lo) <= 1e-12
        assert abs((est["mean"] + est["half"]) - hi) <= 1e-12
        assert abs(est["std"] - statistics.stdev(y.mean(axis=1).tolist())) <= 1e-12
    # identical replications: zero spread, zero half width
    y = np.tile(rng.standard_normal(32), (4, 1))
    est = orc.rqmc(y)
    assert est["std"] == 0.0 and est["half"] == 0.0
