"""GPU parity: every C-ABI entry point against the CPU oracle on the same
seeded inputs, at sizes that span several tiles and passes plus ragged
windows and the degenerate sizes.  Points are compared bit for bit; floating
results normwise against the oracle's long-double twin with the tolerances
stated in each test."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import (F32_EPS, U64_EPS, host_u64, kernel, kernel_scale, pointset, record, rel,
                     solve_tol)

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32


@pytest.fixture(scope="module", autouse=True)
def _init():
    ldk.init()


def _net_or_lattice(kind, seed, m, d, R, nrhs=1, m_max=None):
    if kind == "dnet":
        return W.small_net(seed, m=m, d=d, R=R, nrhs=nrhs, m_max=m_max)
    return W.small_lattice(seed, m=m, d=d, R=R, nrhs=nrhs, m_max=m_max)


# ---------------------------------------------------------------------------
# a1, a2: points (bit-exact)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,order", [("lattice", "natural"), ("lattice", "linear"),
                                        ("dnet", "natural"), ("dnet", "gray")])
@pytest.mark.parametrize("m,d,R", [(0, 3, 1), (1, 1, 2), (5, 4, 3), (10, 33, 2), (13, 70, 1)])
def test_points_bit_exact(orc, kind, order, m, d, R):
    w = _net_or_lattice(kind, 100 + m, m, d, R)
    ps = pointset(w, order)
    n = 2**m
    windows = {(0, n), (n // 2, n), (min(3, n), max(min(3, n), n - 5)), (n // 3, n // 3)}
    for lo, hi in sorted(windows):
        got = host_u64(ldk.gen_points(ps, lo, hi))
        want = orc.points(w, lo, hi, order=order)
        assert got.shape == want.shape
        assert np.array_equal(got, want), (lo, hi)


def test_lattice_natural_beyond_mmax(orc):
    # natural-order lattices are extensible past 2^m_max (Sec. 4.2)
    w = W.small_lattice(5, m=4, d=6, R=2)
    ps = pointset(w)
    got = host_u64(ldk.gen_points(ps, 1000, 1300))
    want = orc.lattice_points(w["gen"], w["shift"], 4, 1000, 1300)
    assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# a3: first Gram column
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("src", ["regen", "pts"])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("order", ["natural", "gray_or_linear"])
def test_kernel_column(orc, kind, src, dtype, order):
    m, d, R = 11, 37, 2
    w = _net_or_lattice(kind, 7, m, d, R)
    if order != "natural":
        w["order"] = "gray" if kind == "dnet" else "linear"
    amax = 4 if kind == "dnet" else 3
    w.update(alpha=np.array([1 + (j % amax) for j in range(d)], np.int32),
             gamma=0.9 ** np.arange(d), zeta=1.3)
    ps, k = pointset(w), kernel(w)
    n = 2**m
    scale = kernel_scale(w)
    tol = (1e-13 if dtype == F64 else 1e-5) * scale
    allpts = orc.points(w)
    for lo, hi in ((0, n), (100, n - 37), (n - 1, n)):
        want = orc.kernel_column(kind, allpts[:, lo:hi], allpts[:, 0], w["alpha"], w["gamma"],
                                 w["zeta"])
        if src == "regen":
            got = ldk.kernel_column(k, ps, lo, hi, dtype=dtype)
        else:
            pts = ldk.gen_points(ps, lo, hi)
            x0 = ldk.gen_points(ps, 0, 1)[:, 0, :].contiguous()
            got = ldk.kernel_column(k, ps, lo, hi, pts=pts, x0=x0, dtype=dtype)
        err = np.max(np.abs(got.cpu().double().numpy() - want))
        assert err <= tol, (lo, hi, err, tol)


@pytest.mark.parametrize("kind,alpha", [("lattice", 1), ("lattice", 2), ("lattice", 3),
                                        ("dnet", 1), ("dnet", 2), ("dnet", 3), ("dnet", 4)])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("order", ["natural", "gray_or_linear"])
def test_kernel_column_uniform_order(orc, kind, alpha, dtype, order):
    # one order for every dimension: the specialised kernels
    m, d, R = 13, 9, 2
    w = _net_or_lattice(kind, 70 + alpha, m, d, R)
    if order != "natural":
        w["order"] = "gray" if kind == "dnet" else "linear"
    w.update(alpha=np.full(d, alpha, np.int32), gamma=0.8 ** np.arange(d), zeta=0.7)
    ps, k = pointset(w), kernel(w)
    n = 2**m
    tol = (1e-13 if dtype == F64 else 1e-5) * kernel_scale(w)
    allpts = orc.points(w)
    for lo, hi in ((0, n), (1000, n - 3000), (2048, 4096), (5, 6)):
        want = orc.kernel_column(kind, allpts[:, lo:hi], allpts[:, 0], w["alpha"], w["gamma"],
                                 w["zeta"])
        got = ldk.kernel_column(k, ps, lo, hi, dtype=dtype)
        err = np.max(np.abs(got.cpu().double().numpy() - want))
        assert err <= tol, (lo, hi, err, tol)


# ---------------------------------------------------------------------------
# a4 building block: the transforms
# ---------------------------------------------------------------------------
TRANSFORM_M = [0, 1, 2, 3, 4, 5, 7, 8, 9, 11, 12, 13, 15, 16, 17, 19, 20, 21]


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", TRANSFORM_M)
@pytest.mark.parametrize("dtype", [F64, F32])
def test_transform(orc, kind, m, dtype):
    n = 2**m
    B = max(1, 2 ** (17 - m)) if m < 17 else 2
    B = min(B, 33) + (m % 3)  # ragged batch counts
    rng = np.random.default_rng(m)
    x = rng.standard_normal((B, n))
    if kind == "lattice":
        x = x + 1j * rng.standard_normal((B, n))
    xd = x.astype(np.complex64 if dtype == F32 else np.complex128) if kind == "lattice" \
        else x.astype(np.float32 if dtype == F32 else np.float64)
    x64 = xd.astype(np.complex128 if kind == "lattice" else np.float64)
    tol = 1e-12 if dtype == F64 else 2e-6
    want = orc.transform(kind, x64, precise=True)
    got = ldk.transform(kind, torch.from_numpy(xd).cuda())
    assert rel(got.cpu().numpy(), want) < tol
    if kind == "lattice":
        back = ldk.transform(kind, torch.from_numpy(xd).cuda(), inverse=True)
        assert rel(back.cpu().numpy(), orc.transform(kind, x64, inverse=True, precise=True)) < tol
    # in place
    t = torch.from_numpy(xd).cuda()
    ldk.transform(kind, t, out=t)
    assert rel(t.cpu().numpy(), want) < tol


# ---------------------------------------------------------------------------
# a4-a6: eig, solve, matvec, logdet on shared inputs
# ---------------------------------------------------------------------------
# lattice rows run as packed half-length complex rows: m = 2, 3 (one pass of
# n/2), 12 / 13 (one or two passes of n/2 in FP64 / FP32), 21 (three passes);
# at m = 20 the passes run the kernels with their tile geometry fixed at
# compile time, the top pass forming the filter itself (one RHS) or reading
# precomputed coefficients (two RHS)
ALG_CASES = [(0, 3), (1, 2), (2, 3), (3, 4), (6, 3), (10, 2), (11, 3), (12, 1), (13, 2),
             (14, 2), (16, 1), (19, 1), (20, 1), (20, 2), (21, 1)]


def _kcol(orc, w):
    pts = orc.points(w)
    return orc.kernel_column(w["kind"], pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"])


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m,nrhs", ALG_CASES)
@pytest.mark.parametrize("dtype", [F64, F32])
def test_eig_solve_matvec_logdet(orc, kind, m, nrhs, dtype):
    d = 6
    R = 2 if m < 16 else 1
    w = _net_or_lattice(kind, 30 + m, m, d, R, nrhs=nrhs)
    w.update(alpha=np.array([2, 1, 3, 2, 1, 2], np.int32), gamma=0.8 ** np.arange(d), zeta=1.0)
    eps = U64_EPS if dtype == F64 else F32_EPS
    np_dt = np.float64 if dtype == F64 else np.float32
    k1 = _kcol(orc, w).astype(np_dt)
    # eig: FP64 transform of the (possibly FP32) column
    lam_ref = orc.eig(kind, k1.astype(np.float64), precise=True)
    lam = ldk.eig(kind, torch.from_numpy(k1).cuda())
    assert lam.dtype == torch.float64
    assert rel(lam.cpu().numpy(), lam_ref) < 1e-12
    # solve / matvec with identical (FP64) lambda on both sides; y, c in dtype
    y = w["y"].astype(np_dt)
    lam_d = torch.from_numpy(lam_ref).cuda()
    for s2 in (1e-2, 1e-8):
        c_ref = orc.solve(kind, lam_ref, s2, y.astype(np.float64), precise=True)
        c = ldk.solve(kind, lam_d, s2, torch.from_numpy(y).cuda())
        tol = max(1e-12 if dtype == F64 else 1e-5, solve_tol(lam_ref, s2, y, c_ref, m, eps))
        err = rel(c.cpu().numpy(), c_ref)
        record(f"solve_{kind}_m{m}_{np_dt.__name__}_s2={s2}", err=err, tol=tol)
        assert err < tol, (s2, err, tol)
    mv_ref = orc.matvec(kind, lam_ref, y.astype(np.float64), precise=True)
    mv = ldk.matvec(kind, lam_d, torch.from_numpy(y).cuda())
    assert rel(mv.cpu().numpy(), mv_ref) < (1e-12 if dtype == F64 else 2e-6)
    # logdet (FP64 throughout)
    ld_ref = orc.logdet(lam_ref, 1e-3, precise=True)
    ld = ldk.logdet(lam_d, 1e-3).cpu().numpy()
    assert np.all(np.abs(ld - ld_ref) <= 1e-12 * np.maximum(1.0, np.abs(ld_ref)) + 2**m * 1e-16)


@pytest.mark.parametrize("kind,m", [("dnet", 14), ("lattice", 14), ("lattice", 9)])
def test_solve_aliasing_and_logdet_nan(orc, kind, m):
    w = _net_or_lattice(kind, 3, m, 4, 1, nrhs=2)
    alpha = [2, 2, 3, 4] if kind == "dnet" else [2, 2, 3, 1]
    w.update(alpha=np.array(alpha, np.int32), gamma=np.ones(4), zeta=1.0)
    k1 = _kcol(orc, w)
    lam = orc.eig(kind, k1, precise=True)
    y = torch.from_numpy(w["y"].copy()).cuda()
    c_ref = orc.solve(kind, lam, 1e-3, w["y"], precise=True)
    ldk.solve(kind, torch.from_numpy(lam).cuda(), 1e-3, y, out=y)  # c overwrites y
    assert rel(y.cpu().numpy(), c_ref) < 1e-12
    bad = lam.copy()
    bad[0, 5] = -1.0
    assert np.isnan(ldk.logdet(torch.from_numpy(bad).cuda(), 1e-3).cpu().numpy()[0])


# ---------------------------------------------------------------------------
# a7: transform and eigenvalue updates (n -> 2n)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 4, 10, 11, 12, 13, 17, 19])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_update_double(orc, kind, m, dtype):
    n = 2**m
    B = 3 if m < 17 else 1
    rng = np.random.default_rng(m)
    np_dt = np.float64 if dtype == F64 else np.float32
    y_old = rng.standard_normal((B, n)).astype(np_dt)
    y_new = rng.standard_normal((B, n)).astype(np_dt)
    cdt = np.complex128 if dtype == F64 else np.complex64
    if kind == "lattice":
        yt_old = orc.transform(kind, y_old.astype(np.complex128), precise=True).astype(cdt)
        fresh = orc.transform(kind, np.concatenate([y_old, y_new], 1).astype(np.complex128),
                              precise=True)
    else:
        yt_old = orc.transform(kind, y_old.astype(np.float64), precise=True).astype(np_dt)
        fresh = orc.transform(kind, np.concatenate([y_old, y_new], 1).astype(np.float64),
                              precise=True)
    got = ldk.update_double(kind, torch.from_numpy(yt_old).cuda(), torch.from_numpy(y_new).cuda())
    assert rel(got.cpu().numpy(), fresh) < (1e-12 if dtype == F64 else 2e-6)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 5, 11, 12, 13, 18])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_eig_update_double(orc, kind, m, dtype):
    d = 5
    w = _net_or_lattice(kind, 50 + m, m + 1, d, 2)
    w.update(alpha=np.array([2, 3, 1, 2, 2], np.int32), gamma=0.7 ** np.arange(d), zeta=1.0)
    np_dt = np.float64 if dtype == F64 else np.float32
    k1 = _kcol(orc, w).astype(np_dt)
    n = 2**m
    lam_half = orc.eig(kind, k1[:, :n].astype(np.float64), precise=True)
    fresh = orc.eig(kind, k1.astype(np.float64), precise=True)
    got = ldk.eig_update_double(kind, torch.from_numpy(lam_half).cuda(),
                                torch.from_numpy(np.ascontiguousarray(k1[:, n:])).cuda())
    assert got.dtype == torch.float64
    assert rel(got.cpu().numpy(), fresh) < 1e-12
