"""Higher-order nets (Sec. 4.3, digital interlacing with higher-order LMS) on
the GPU against the oracle: the interlaced scrambled columns and the points
bit for bit, and the first Gram column and its gradient on those points
(regenerated from the per-replication columns) within the kernel-column
tolerances."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import dev_u64, host_u64, kernel_scale

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32


@pytest.fixture(scope="module", autouse=True)
def _init():
    ldk.init()


def _src(alpha, seed, m, d, R, lms=True):
    """Source net of alpha d dimensions (shared columns, per-replication scrambles)."""
    w = W.small_net(seed, m=m, d=alpha * d, R=R)
    if not lms:
        w["lms"] = None
    ps = ldk.PointSet("dnet", R, alpha * d, m, dev_u64(w["gen"]),
                      None if w["lms"] is None else dev_u64(w["lms"]), None)
    rng = np.random.default_rng(seed + 1000)
    shift = rng.integers(0, 2**63, size=(R, d), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(R, d), dtype=np.uint64)
    return w, ps, shift


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
@pytest.mark.parametrize("m,d,R", [(0, 2, 1), (1, 1, 2), (6, 3, 2), (13, 16, 2)])
@pytest.mark.parametrize("lms", [True, False])
def test_interlaced_columns(orc, alpha, m, d, R, lms):
    w, ps, _ = _src(alpha, 50 + m + alpha, m, d, R, lms)
    hp = ldk.interlace(ps, alpha)
    want = orc.interlace_columns(w["gen"], w["lms"], alpha, R)
    assert np.array_equal(host_u64(hp.gen), want.reshape(R, d, m))


@pytest.mark.parametrize("alpha", [2, 3, 4])
@pytest.mark.parametrize("order", ["natural", "gray"])
def test_higher_order_points(orc, alpha, order):
    m, d, R = 12, 5, 2
    w, ps, shift = _src(alpha, 60 + alpha, m, d, R)
    hp = ldk.interlace(ps, alpha, shift=dev_u64(shift), order=order)
    n = 2**m
    for lo, hi in ((0, n), (37, n - 100), (n - 1, n)):
        got = host_u64(ldk.gen_points(hp, lo, hi))
        want = orc.higher_order_dnet_points(w["gen"], w["lms"], shift, alpha, m, lo, hi, order)
        assert np.array_equal(got, want), (lo, hi)


@pytest.mark.parametrize("alpha", [2, 3, 4])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_higher_order_kernel_column(orc, alpha, dtype):
    # the order-alpha DSI kernel on the order-alpha net, points regenerated
    m, d, R = 13, 6, 2
    w, ps, shift = _src(alpha, 70 + alpha, m, d, R)
    hp = ldk.interlace(ps, alpha, shift=dev_u64(shift))
    gamma = 0.8 ** np.arange(d)
    k = ldk.Kernel("dnet", np.full(d, alpha, np.int32), torch.from_numpy(gamma).cuda(), 1.2)
    n = 2**m
    pts = orc.higher_order_dnet_points(w["gen"], w["lms"], shift, alpha, m, 0, n)
    scale = kernel_scale({"kind": "dnet", "alpha": np.full(d, alpha), "gamma": gamma, "zeta": 1.2})
    tol = (1e-13 if dtype == F64 else 1e-5) * scale
    for lo, hi in ((0, n), (1000, n - 3000)):
        want = orc.kernel_column("dnet", pts[:, lo:hi], pts[:, 0], np.full(d, alpha, np.int32),
                                 gamma, 1.2)
        got = ldk.kernel_column(k, hp, lo, hi, dtype=dtype).cpu().double().numpy()
        assert np.max(np.abs(got - want)) <= tol, (lo, hi)
        # points_column runs the same two calls for nets: the same outputs
        p2, k2 = ldk.points_column(k, hp, lo, hi, dtype=dtype)
        assert np.array_equal(host_u64(p2), pts[:, lo:hi])
        assert torch.equal(k2, ldk.kernel_column(k, hp, lo, hi, dtype=dtype))


def test_higher_order_kernel_grad(orc):
    alpha, m, d, R = 2, 12, 5, 2
    w, ps, shift = _src(alpha, 81, m, d, R)
    hp = ldk.interlace(ps, alpha, shift=dev_u64(shift))
    gamma = 0.7 ** np.arange(1, d + 1)
    al = np.full(d, alpha, np.int32)
    k = ldk.Kernel("dnet", al, torch.from_numpy(gamma).cuda(), 0.9)
    n = 2**m
    pts = orc.higher_order_dnet_points(w["gen"], w["lms"], shift, alpha, m, 0, n)
    a = np.random.default_rng(5).standard_normal((R, n))
    want = orc.kernel_grad("dnet", pts, pts[:, 0], al, gamma, 0.9, a)
    got = ldk.kernel_grad(k, hp, 0, n, torch.from_numpy(a).cuda()).cpu().numpy()
    bound = np.abs(a).sum(axis=1, keepdims=True) * kernel_scale(
        {"kind": "dnet", "alpha": al, "gamma": gamma, "zeta": 0.9})
    assert np.max(np.abs(got - want) / bound) < 1e-14
