"""Pins for the oracle's Gram algebra (Sec. 5.2-5.4): structure, eigenvalues,
solve and log-det against dense brute force, CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import brute
from golden_io import frac, rows


def _with_kernel(w, alpha, gamma, zeta=1.0):
    w = dict(w)
    w.update(alpha=np.asarray(alpha, np.int32), gamma=np.asarray(gamma, float), zeta=zeta)
    return w


def _dense(orc, w, pts):
    """Dense Gram from the points pairwise: column l is the kernel column
    anchored at point l."""
    R, n, d = pts.shape
    K = np.empty((R, n, n))
    for r in range(R):
        for l in range(n):
            K[r, :, l] = orc.kernel_column(w["kind"], pts[r:r + 1], pts[r:r + 1, l], w["alpha"],
                                           w["gamma"], w["zeta"])[0]
    return K


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_net_gram_is_rsbt(orc, alpha):
    # Sec. 5.3: digitally shifted (LMS) net in natural order x DSI kernel:
    # K[i, l] = k1[i XOR l] exactly, since x_i (-) x_l = z_{i XOR l}
    w = _with_kernel(W.small_net(alpha, m=6, d=3, R=2), [alpha] * 3, [1.0, 0.7, 0.3], 1.3)
    pts = orc.points(w)
    K = _dense(orc, w, pts)
    k1 = K[:, :, 0]
    n = 64
    idx = np.arange(n)
    for r in range(2):
        np.testing.assert_array_equal(K[r], k1[r][idx[:, None] ^ idx[None, :]])


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_lattice_gram_is_circulant(orc, alpha):
    # Sec. 5.2: shifted lattice in linear order x SI kernel is circulant
    w = _with_kernel(W.small_lattice(alpha, m=6, d=3, R=1), [alpha] * 3, [1.0, 0.5, 0.2])
    lin = orc.points(w, order="linear")
    K = _dense(orc, w, lin)[0]
    n = 64
    for a in range(n):
        for b in range(n):
            assert K[a, b] == K[(a - b) % n, 0]
    # natural order: K[i, l] = c[(R(i) - R(l)) mod n] with c the linear-order column
    nat = orc.points(w)
    Kn = _dense(orc, w, nat)[0]
    R_ = [brute.bitrev(i, 6) for i in range(n)]
    for i in range(n):
        for l in range(n):
            assert Kn[i, l] == K[(R_[i] - R_[l]) % n, 0]


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_eigendecomposition_reconstructs_gram(orc, kind):
    # Sec. 5.4: K = V Lambda conj(V), lambda = sqrt(n) conj(V) k1
    m, n = 6, 64
    base = W.small_lattice(2, m=m, d=4) if kind == "lattice" else W.small_net(2, m=m, d=4)
    w = _with_kernel(base, [2, 1, 3, 2], [1.0, 0.5, 0.25, 0.125])
    pts = orc.points(w)
    K = _dense(orc, w, pts)[0]
    lam, max_imag = orc.eig(kind, K[None, :, 0])
    assert max_imag < 1e-12 * np.abs(lam).max()
    V = (brute.fourier_br(m).conj().T if kind == "lattice" else brute.hadamard(m)) / math.sqrt(n)
    np.testing.assert_allclose(V @ np.diag(lam[0]) @ V.conj().T, K, atol=1e-12 * np.abs(K).max())
    assert lam.min() > 0  # positive Walsh / Fourier coefficients


def test_worked_examples_n4(orc):
    g = {r[0]: r[1:] for r in rows("eig_worked_n4.txt")}
    # net: van der Corput, 1 + K_2
    C = np.array([[1 << 63, 1 << 62]], dtype=np.uint64)
    pts = orc.dnet_points(C, None, None, 2, 0, 4, R=1)
    k1 = orc.kernel_column("dnet", pts, pts[:, 0], [2], [1.0], 1.0)
    np.testing.assert_array_equal(k1[0], [float(frac(v)) for v in g["net_k1"]])
    lam, _ = orc.eig("dnet", k1)
    np.testing.assert_allclose(lam[0], [float(frac(v)) for v in g["net_lambda"]], atol=1e-15)
    for k in range(4):
        assert abs(4 * brute.net_alias_sum(2, k, 2) - frac(g["net_lambda"][k])) < Fraction(1, 10**18)
    # lattice: g = 1, 1 + K_1
    pts = orc.lattice_points(np.array([1], np.uint64), None, 2, 0, 4)
    k1 = orc.kernel_column("lattice", pts, pts[:, 0], [1], [1.0], 1.0)
    lam, _ = orc.eig("lattice", k1)
    want = [float(frac(a)) + float(frac(b)) * math.pi**2
            for a, b in (v.split(",") for v in g["lattice_lambda_pi2"])]
    np.testing.assert_allclose(lam[0], want, atol=1e-14)


@pytest.mark.parametrize("alpha", [2, 3, 4])
@pytest.mark.parametrize("m", [3, 4])
def test_net_eig_equals_walsh_aliasing(orc, alpha, m):
    # d = 1 van der Corput net: lambda_k = n sum_{h == k mod n} r(h)
    n = 2**m
    C = np.array([[1 << (63 - k) for k in range(m)]], dtype=np.uint64)
    pts = orc.dnet_points(C, None, None, m, 0, n, R=1)
    k1 = orc.kernel_column("dnet", pts, pts[:, 0], [alpha], [1.0], 1.0)
    lam, _ = orc.eig("dnet", k1)
    want = [float(n * brute.net_alias_sum(alpha, k, m)) for k in range(n)]
    np.testing.assert_allclose(lam[0], want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("alpha", [1, 2, 3])
@pytest.mark.parametrize("m", [3, 6])
def test_lattice_eig_equals_fourier_aliasing(orc, alpha, m):
    # d = 1, g = 1: lambda_k = n sum_{h == k mod n} c(h)
    n = 2**m
    pts = orc.lattice_points(np.array([1], np.uint64), None, m, 0, n)
    k1 = orc.kernel_column("lattice", pts, pts[:, 0], [alpha], [1.0], 1.0)
    lam, _ = orc.eig("lattice", k1)
    want = [n * brute.lattice_alias_sum(alpha, k, n) for k in range(n)]
    np.testing.assert_allclose(lam[0], want, rtol=1e-12, atol=1e-12)


def _dense_check(orc, w, nrhs=2):
    pts = orc.points(w)
    K = _dense(orc, w, pts)
    lam, _ = orc.eig(w["kind"], K[:, :, 0])
    rng = np.random.default_rng(0)
    y = rng.standard_normal((w["R"], nrhs, K.shape[1]))
    s2 = w["sigma2"]
    c = orc.solve(w["kind"], lam, s2, y)
    mv = orc.matvec(w["kind"], lam, y)
    ld = orc.logdet(lam, s2)
    for r in range(w["R"]):
        Ks = K[r] + s2 * np.eye(K.shape[1])
        L = np.linalg.cholesky(Ks)
        cd = np.linalg.solve(L.T, np.linalg.solve(L, y[r].T)).T
        cond = np.linalg.cond(Ks)
        err = np.linalg.norm(c[r] - cd) / np.linalg.norm(cd)
        assert err < 50 * cond * 2.0**-53, (err, cond)
        np.testing.assert_allclose(mv[r], (K[r] @ y[r].T).T, atol=1e-12 * np.abs(K[r]).sum(1).max())
        ldd = 2 * np.sum(np.log(np.diag(L)))
        assert abs(ld[r] - ldd) < 1e-11 * max(1, abs(ldd)) + 50 * cond * 2.0**-53
    return c


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_solve_logdet_match_dense_cholesky(orc, kind):
    base = W.small_lattice(9, m=7, d=3, R=2) if kind == "lattice" else W.small_net(9, m=7, d=3, R=2)
    w = _with_kernel(base, [2, 2, 1], [1.0, 0.5, 0.3])
    w["sigma2"] = 1e-3
    _dense_check(orc, w)


@pytest.mark.slow
def test_workload1_full_dense(orc):
    # order-1 DSI kernel, n = 1024, d = 4, sigma^2 = 1e-8: dense Gram + Cholesky
    _dense_check(orc, W.workload(1), nrhs=1)


def test_logdet_flags_nonpositive(orc):
    lam = np.array([[1.0, 0.5, -0.2, 2.0]])
    out = orc.logdet(lam, 0.1)
    assert np.isnan(out[0])
