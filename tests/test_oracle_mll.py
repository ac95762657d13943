"""Pins of the oracle's GP marginal likelihood and gradient (CPU only).

The fast oracle works in the eigenbasis of Sec. 5.4 (transforms of y and of
dL/dlambda, prefix/suffix products over the dimensions); every pin below
reaches the same numbers by another route:
  * the dense GP log-likelihood and its trace-form gradient
        dL/dtheta = 1/2 c^T (dK/dtheta) c - 1/2 tr((K + s2 I)^-1 dK/dtheta)
    with a dense Gram built pairwise and numpy's solve / slogdet;
  * central differences of the oracle's own objective;
  * the adjoint identity <g, lambda(v)> = <a(g), v> for the linear map
    v -> lambda = sqrt(n) FT(v);
  * a factor 1 + gamma K that is exactly zero (DSI order 1 at x >= 1/2 with
    gamma = 2), where dividing the product by the factor would give NaN.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _inst(kind, seed, m, d, R, alpha, gamma, zeta=1.0, sigma2=1e-2):
    w = W.small_lattice(seed, m, d, R) if kind == "lattice" else W.small_net(seed, m, d, R)
    w.update(alpha=np.array(alpha, np.int32), gamma=np.array(gamma, np.float64), zeta=zeta,
             sigma2=sigma2)
    return w


def _pair_factors(kind, alpha, pts_r):
    """F[j][a][b] = K_{alpha_j}(x_a (-) x_b) for one replication (pairwise)."""
    n, d = pts_r.shape
    F = np.empty((d, n, n))
    for j in range(d):
        u = pts_r[:, j]
        for a in range(n):
            for b in range(n):
                if kind == "lattice":
                    F[j, a, b] = O.si_factor(int(alpha[j]), (int(u[a]) - int(u[b])) % 2**64)
                else:
                    F[j, a, b] = O.dsi_factor(int(alpha[j]), int(u[a]) ^ int(u[b]))
    return F


def _dense(w, y):
    """Dense GP objective and gradient per replication."""
    pts = O.points(w)
    R, n, d = pts.shape
    gamma, zeta, s2 = w["gamma"], w["zeta"], w["sigma2"]
    Ls, grads = [], []
    for r in range(R):
        F = _pair_factors(w["kind"], w["alpha"], pts[r])
        fac = 1.0 + gamma[:, None, None] * F
        K = zeta * np.prod(fac, axis=0)
        dK = []
        for j in range(d):
            others = np.prod(np.delete(fac, j, axis=0), axis=0)
            dK.append(zeta * gamma[j] * F[j] * others)
        dK.append(K)  # log zeta
        dK.append(s2 * np.eye(n))  # log sigma2
        Ks = K + s2 * np.eye(n)
        c = np.linalg.solve(Ks, y[r])
        sign, ld = np.linalg.slogdet(Ks)
        assert sign > 0
        Ls.append(-0.5 * y[r] @ c - 0.5 * ld - 0.5 * n * math.log(2 * math.pi))
        Ki = np.linalg.inv(Ks)
        grads.append([0.5 * c @ D @ c - 0.5 * np.sum(Ki * D.T) for D in dK])
    return np.array(Ls), np.array(grads)


CASES = [("lattice", [2, 1, 3]), ("dnet", [2, 4, 1])]


@pytest.mark.parametrize("kind,alpha", CASES)
def test_mll_and_gradient_match_dense_gp(kind, alpha):
    w = _inst(kind, 11, 6, 3, 2, alpha, [0.9, 0.5, 0.3], zeta=1.3, sigma2=2e-2)
    y = w["y"][:, 0, :]
    fast = O.mll_grad(w)
    L, G = _dense(w, y)
    assert np.allclose(fast["L"], L, rtol=1e-10, atol=1e-10), (fast["L"], L)
    scale = np.abs(G).max()
    assert np.abs(fast["grad"] - G).max() <= 1e-9 * scale, (fast["grad"], G)


@pytest.mark.parametrize("kind,alpha", CASES)
def test_gradient_central_differences(kind, alpha):
    m, d = 10, 3
    w = _inst(kind, 12, m, d, 1, alpha, [0.8, 0.6, 0.4], zeta=0.7, sigma2=5e-3)
    theta = np.concatenate([np.log(w["gamma"]), [math.log(w["zeta"]), math.log(w["sigma2"])]])

    def L(th):
        return O.mll_grad(w, gamma=np.exp(th[:d]), zeta=math.exp(th[d]),
                          sigma2=math.exp(th[d + 1]))["L"][0]

    grad = O.mll_grad(w)["grad"][0]
    h = 1e-5
    fd = np.empty(d + 2)
    for p in range(d + 2):
        e = np.zeros(d + 2)
        e[p] = h
        fd[p] = (L(theta + e) - L(theta - e)) / (2 * h)
    # central differences: O(h^2) truncation plus |L| eps / h rounding
    tol = 1e-6 * max(1.0, np.abs(grad).max()) + 1e-16 * abs(L(theta)) / h * 10
    assert np.abs(fd - grad).max() <= tol, (fd, grad)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 3, 7])
def test_adjoint_dot_product(kind, m):
    """<g, lambda(v)> == <adjoint(g), v> for the linear map v -> sqrt(n) Re FT(v)."""
    rng = np.random.default_rng(100 + m)
    n = 2**m
    v = rng.standard_normal((2, n))
    g = rng.standard_normal((2, n))  # not symmetric: the Re of the lattice map matters
    lam = O.eig(kind, v)[0]
    a = O.mll_adjoint(kind, g)
    assert np.allclose(np.sum(g * lam, axis=1), np.sum(a * v, axis=1), rtol=1e-12, atol=1e-12)


def test_gradient_through_an_exactly_zero_factor():
    """DSI order 1: K_1(x) = -1/2 on [1/2, 1), so gamma = 2 zeroes the factor."""
    w = _inst("dnet", 13, 6, 2, 1, [1, 2], [2.0, 0.5], zeta=1.0, sigma2=5e-2)
    pts = O.points(w)
    x0 = pts[:, 0, :]
    zero = [O.dsi_factor(1, int(u) ^ int(x0[0, 0])) * 2.0 + 1.0 for u in pts[0, :, 0]]
    assert min(abs(z) for z in zero) == 0.0  # the case is really hit
    fast = O.mll_grad(w)
    assert np.all(np.isfinite(fast["grad"]))
    L, G = _dense(w, w["y"][:, 0, :])
    assert np.abs(fast["grad"] - G).max() <= 1e-9 * np.abs(G).max()
    assert np.allclose(fast["L"], L, rtol=1e-10)


def test_mll_sigma_derivative_and_constant():
    """With lambda = 0 the objective is that of white noise s2 I:
    L = -|y|^2 / (2 s2) - n/2 log s2 - n/2 log 2 pi, dL/dlog s2 = |y|^2/(2 s2) - n/2."""
    rng = np.random.default_rng(7)
    for kind in ("lattice", "dnet"):
        y = rng.standard_normal((3, 16))
        s2 = 0.37
        L, g, ds = O.mll(kind, np.zeros((3, 16)), s2, y)
        yy = np.sum(y * y, axis=1)
        assert np.allclose(L, -yy / (2 * s2) - 8 * math.log(s2) - 8 * math.log(2 * math.pi),
                           rtol=1e-13)
        assert np.allclose(ds, yy / (2 * s2) - 8, rtol=1e-12)


def _pair_factors_by_columns(kind, alpha, pts_r):
    """F[j][a][b] = K_{alpha_j}(x_a (-) x_b), column b at a time: the
    one-dimensional kernel column anchored at point b with gamma = zeta = 1
    is 1 + K_{alpha_j}(x_a (-) x_b)."""
    n, d = pts_r.shape
    F = np.empty((d, n, n))
    for j in range(d):
        col = np.ascontiguousarray(pts_r[None, :, j:j + 1])
        for b in range(n):
            F[j, :, b] = O.kernel_column(kind, col, col[:, b, :], [int(alpha[j])], [1.0],
                                         1.0)[0] - 1.0
    return F


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_gradient_dense_at_n256_d64(kind):
    """The gradient workload's dense check: n = 2^8, d = 64 (order-2 kernel,
    gamma_j = 1/j^2, sigma2 = 1e-3), dense Gram and the trace-form gradient
    against the eigenbasis gradient.  Tolerance from the conditioning: the
    dense solve and inverse carry about kappa u with
    kappa = (lambda_max + s2) / (lambda_min + s2)."""
    m, d = 8, 64
    w = _inst(kind, 64, m, d, 1, [2] * d, 1.0 / np.arange(1, d + 1) ** 2, zeta=1.0, sigma2=1e-3)
    y = w["y"][:, 0, :]
    fast = O.mll_grad(w)
    pts = O.points(w)
    n = 2**m
    F = _pair_factors_by_columns(kind, w["alpha"], pts[0])
    fac = 1.0 + w["gamma"][:, None, None] * F
    K = w["zeta"] * np.prod(fac, axis=0)
    s2 = w["sigma2"]
    Ks = K + s2 * np.eye(n)
    c = np.linalg.solve(Ks, y[0])
    Ki = np.linalg.inv(Ks)
    sign, ld = np.linalg.slogdet(Ks)
    assert sign > 0
    L = -0.5 * y[0] @ c - 0.5 * ld - 0.5 * n * math.log(2 * math.pi)
    G = []
    # prefix / suffix products of the factors (no division by a factor)
    pre = np.ones((d + 1, n, n))
    for j in range(d):
        pre[j + 1] = pre[j] * fac[j]
    suf = np.ones((n, n))
    dK = [None] * d
    for j in range(d - 1, -1, -1):
        dK[j] = w["zeta"] * w["gamma"][j] * F[j] * pre[j] * suf
        suf = suf * fac[j]
    dK += [K, s2 * np.eye(n)]
    T1 = np.array([0.5 * c @ D @ c for D in dK])
    T2 = np.array([0.5 * np.sum(Ki * D.T) for D in dK])
    G = T1 - T2
    lam = np.linalg.eigvalsh(Ks)
    kappa = lam.max() / lam.min()
    u = 2.0**-53
    # each trace-form term carries the dense solve's / inverse's relative
    # error (backward stable: about n u kappa) on its own magnitude, and G is
    # their difference; the eigenbasis side is far more accurate
    scale_t = np.abs(T1) + 0.5 * np.linalg.norm(Ki) * np.array([np.linalg.norm(D) for D in dK])
    tol_g = 4 * n * u * kappa * scale_t
    tol_L = 4 * n * u * kappa * (abs(L) + abs(y[0] @ c))
    assert abs(fast["L"][0] - L) <= tol_L, (fast["L"][0], L, tol_L)
    err = np.abs(fast["grad"][0] - G)
    assert np.all(err <= tol_g), (np.max(err / tol_g), err[np.argmax(err / tol_g)])


@pytest.mark.parametrize("kind,alpha", CASES)
def test_gradient_central_differences_h1e6(kind, alpha):
    """Central differences with the step the gradient workload states
    (h = 1e-6).  Tolerance: twice the O(h^2) truncation estimated from the
    same difference at 2h (FD(2h) - FD(h) = 3 c h^2), plus the objective's
    rounding 8 (m + 4) u |L| on each evaluation, divided by 2h."""
    m, d = 10, 3
    w = _inst(kind, 12, m, d, 1, alpha, [0.8, 0.6, 0.4], zeta=0.7, sigma2=5e-3)
    theta = np.concatenate([np.log(w["gamma"]), [math.log(w["zeta"]), math.log(w["sigma2"])]])

    def L(th):
        return O.mll_grad(w, gamma=np.exp(th[:d]), zeta=math.exp(th[d]),
                          sigma2=math.exp(th[d + 1]))["L"][0]

    grad = O.mll_grad(w)["grad"][0]
    h = 1e-6
    rnd = 8 * (m + 4) * 2.0**-53 * abs(L(theta))
    for p in range(d + 2):
        e = np.zeros(d + 2)
        e[p] = h
        fd1 = (L(theta + e) - L(theta - e)) / (2 * h)
        fd2 = (L(theta + 2 * e) - L(theta - 2 * e)) / (4 * h)
        tol = 2 * abs(fd2 - fd1) / 3 + 2 * rnd / (2 * h) + 2 * rnd / (4 * h)
        assert abs(fd1 - grad[p]) <= tol, (p, fd1, grad[p], tol)
