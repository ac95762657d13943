"""Pins for the oracle's kernel cubature (Sec. 3.2): the
squared worst-case error against closed forms for equal weights in one
dimension, the mean-zero property of every kernel factor behind
kappa_i = zeta, optimality of the weights, and the Bayesian-cubature
posterior on functions in the span of the kernel.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import brute

ZETA, GAMMA = 1.7, 0.6


def _d1(kind, m, alpha, seed):
    """One-dimensional instance: the lattice with g = 1 (points j / n + shift)
    or the digital net with the identity generating matrix (the dyadic grid
    (+) shift), a random shift either way."""
    rng = np.random.default_rng(seed)
    shift = rng.integers(0, 2**64, size=(1, 1), dtype=np.uint64)
    if kind == "lattice":
        w = dict(kind="lattice", m=m, d=1, R=1, gen=np.array([1], np.uint64), lms=None,
                 shift=shift)
    else:
        C = np.array([[np.uint64(1) << np.uint64(63 - k) for k in range(m)]], np.uint64)
        w = dict(kind="dnet", m=m, d=1, R=1, gen=C, lms=None, shift=shift)
    w.update(alpha=np.array([alpha], np.int32), gamma=np.array([GAMMA]), zeta=ZETA)
    return w


def _equal(n):
    return np.full((1, 1, n), 1.0 / n)


@pytest.mark.parametrize("alpha,m", [(1, 2), (1, 4), (1, 6), (2, 2), (2, 3), (2, 4), (3, 2),
                                     (3, 3)])
def test_lattice_equal_weights_closed_form(orc, alpha, m):
    # equal weights on {j/n + shift}: e^2 = zeta gamma (mean of K_alpha over
    # the n points) = zeta gamma sum_{h != 0, n | h} |h|^{-2 alpha}
    #          = zeta gamma 2 zeta_R(2 alpha) / n^{2 alpha}
    n = 2**m
    w = _d1("lattice", m, alpha, seed=10 * alpha + m)
    K = orc.gram("lattice", orc.points(w), w["alpha"], w["gamma"], ZETA)
    kappa, I2 = orc.kernel_integrals(ZETA, n)
    e2 = orc.wce2(K, kappa, I2, _equal(n))[0, 0]
    exact = ZETA * GAMMA * (brute.lattice_alias_sum(alpha, 0, n) - 1.0)
    assert abs(e2 - exact) <= 1e-12 + 1e-9 * exact
    assert e2 > 0


@pytest.mark.parametrize("alpha,m", [(2, 2), (2, 4), (2, 6), (3, 3), (3, 5), (4, 2), (4, 4)])
def test_net_equal_weights_closed_form(orc, alpha, m):
    # equal weights on the dyadic grid (+) shift: e^2 = zeta gamma (mean of
    # K_alpha over the grid) = zeta gamma sum_{h >= 1, 2^m | h} r_alpha(h)
    n = 2**m
    w = _d1("dnet", m, alpha, seed=10 * alpha + m)
    K = orc.gram("dnet", orc.points(w), w["alpha"], w["gamma"], ZETA)
    kappa, I2 = orc.kernel_integrals(ZETA, n)
    e2 = orc.wce2(K, kappa, I2, _equal(n))[0, 0]
    exact = ZETA * GAMMA * float(brute.net_alias_sum(alpha, 0, m) - 1)
    assert abs(e2 - exact) <= 1e-12 + 1e-9 * exact
    assert e2 > 0


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_si_factor_mean_zero(orc, alpha):
    # kappa_i = zeta needs int_0^1 K_alpha(u - x) du = 0: the mean over a
    # shifted grid of N points is the aliased Fourier sum, |.| <= 2 zeta_R(2a)/N^2a
    N = 2**12
    rng = np.random.default_rng(alpha)
    for x in rng.integers(0, 2**64, size=4, dtype=np.uint64):
        vals = [orc.si_factor(alpha, (int(g) * 2**52 - int(x)) % 2**64) for g in range(N)]
        bound = brute.lattice_alias_sum(alpha, 0, N) - 1.0
        assert abs(np.mean(vals)) <= bound + 1e-14


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_dsi_factor_mean_zero(orc, alpha):
    # the DSI factor over the dyadic grid (+) x: the Walsh series keeps the
    # frequencies that are multiples of N, all with positive coefficients
    N, logN = 2**12, 12
    rng = np.random.default_rng(10 + alpha)
    bound = float(brute.net_alias_sum(max(alpha, 2), 0, logN) - 1) if alpha > 1 else 2.0**-12
    for x in rng.integers(0, 2**64, size=4, dtype=np.uint64):
        vals = [orc.dsi_factor(alpha, (g << 52) ^ int(x)) for g in range(N)]
        assert abs(np.mean(vals)) <= bound + 1e-14


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_optimal_weights(orc, kind):
    # Sec. 3.2: omega* = K^{-1} kappa minimises e^2; the
    # points form a group, so the constant vector is an eigenvector of K with
    # eigenvalue sum_i k1_i and all weights equal zeta / sum_i k1_i
    m, n = 6, 64
    base = W.small_lattice(3, m=m, d=3) if kind == "lattice" else W.small_net(3, m=m, d=3)
    w = dict(base, alpha=np.array([2, 1, 3], np.int32), gamma=np.array([1.0, 0.4, 0.2]),
             zeta=ZETA)
    K = orc.gram(kind, orc.points(w), w["alpha"], w["gamma"], ZETA)
    kappa, I2 = orc.kernel_integrals(ZETA, n)
    bc = orc.bayes_cubature(K, kappa, I2, w["y"][:, 0, :], 0.0)
    ws = bc["weights"]
    np.testing.assert_allclose(ws[0], ZETA / K[0, :, 0].sum(), rtol=1e-9)
    e_opt = orc.wce2(K, kappa, I2, ws[:, None, :])[0, 0]
    e_eq = orc.wce2(K, kappa, I2, _equal(n))[0, 0]
    assert 0.0 <= e_opt <= e_eq
    # stationarity: e^2(w* + t d) = e^2(w*) + t^2 d^T K d (no linear term)
    rng = np.random.default_rng(7)
    for _ in range(3):
        d = rng.standard_normal(n) / n
        ep = orc.wce2(K, kappa, I2, (ws + d)[:, None, :])[0, 0]
        em = orc.wce2(K, kappa, I2, (ws - d)[:, None, :])[0, 0]
        quad = d @ K[0] @ d
        assert abs((ep - em) / 2) <= 1e-10 * (quad + e_opt)
        assert abs((ep + em) / 2 - e_opt - quad) <= 1e-10 * (quad + e_opt)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_bayes_cubature_exact_on_kernel_sections(orc, kind):
    # f = K(., x_l) lies in the span: with sigma2 = 0 the posterior mean is
    # its integral kappa_l = zeta exactly, and y^T K^{-1} y = K_ll
    m, n = 5, 32
    base = W.small_lattice(5, m=m, d=2) if kind == "lattice" else W.small_net(5, m=m, d=2)
    w = dict(base, alpha=np.array([1, 2], np.int32), gamma=np.array([0.8, 0.5]), zeta=ZETA)
    K = orc.gram(kind, orc.points(w), w["alpha"], w["gamma"], ZETA)
    kappa, I2 = orc.kernel_integrals(ZETA, n)
    for l in (0, 3, n - 1):
        bc = orc.bayes_cubature(K, kappa, I2, K[:, :, l], 0.0)
        assert abs(bc["mean"][0] - ZETA) <= 1e-9
        assert abs(bc["s2"][0] - K[0, l, l] / n) <= 1e-9 * K[0, l, l] / n
        # posterior variance of the integral = squared WCE of the optimal weights
        assert abs(bc["var"][0] - bc["wce2"][0]) <= 1e-10 * ZETA
        assert bc["var"][0] >= 0


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("sigma2", [0.0, 1e-3])
def test_fast_equals_dense(orc, kind, sigma2):
    # the eigenvalue (Sec. 5.4) forms agree with the dense definitions
    m, n, R, nw = 6, 64, 2, 3
    base = (W.small_lattice(9, m=m, d=4, R=R) if kind == "lattice"
            else W.small_net(9, m=m, d=4, R=R))
    w = dict(base, alpha=np.array([2, 2, 1, 3], np.int32),
             gamma=np.array([1.0, 0.5, 0.25, 0.125]), zeta=ZETA)
    pts = orc.points(w)
    K = orc.gram(kind, pts, w["alpha"], w["gamma"], ZETA)
    kappa, I2 = orc.kernel_integrals(ZETA, n)
    lam, _ = orc.eig(kind, K[:, :, 0])
    om = W.cubature_weights(4, R, nw, n)
    np.testing.assert_allclose(orc.wce2_fast(kind, lam, ZETA, om), orc.wce2(K, kappa, I2, om),
                               rtol=1e-9, atol=1e-12)
    y = w["y"][:, 0, :]
    fast = orc.bayes_cubature_fast(kind, lam, sigma2, ZETA, y)
    dense = orc.bayes_cubature(K, kappa, I2, y, sigma2)
    for key in ("mean", "var", "s2", "wce2"):
        np.testing.assert_allclose(fast[key], dense[key], rtol=1e-7, atol=1e-11, err_msg=key)
    np.testing.assert_allclose(fast["weights"], dense["weights"], rtol=1e-7)
