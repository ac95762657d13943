"""GPU parity on the named workloads at their full sizes, with the C ABI
called exactly as the benchmark calls it.  Points are compared bit for bit
over the whole set; k1, lambda, c and the log-det against the oracle."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import (F32_EPS, U64_EPS, dev_u64, host_u64, kernel, kernel_scale, pointset, rel,
                     solve_tol)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _init():
    ldk.init()


def _fit_on_gpu(w, y, dtype):
    ps, k = pointset(w), kernel(w)
    n = 2 ** w["m"]
    pts = ldk.gen_points(ps, 0, n)
    k1 = ldk.kernel_column(k, ps, 0, n, dtype=dtype)
    lam = ldk.eig(w["kind"], k1)
    c = ldk.solve(w["kind"], lam, w["sigma2"], y.to(dtype))
    ld = ldk.logdet(lam, w["sigma2"])
    torch.cuda.synchronize()
    return pts, k1, lam, c, ld


def _check(orc, w, y_host, dtype=torch.float64):
    ref = orc.fit_solve(w, y=y_host, precise=True)
    pts, k1, lam, c, ld = _fit_on_gpu(w, torch.from_numpy(y_host).cuda(), dtype)
    assert np.array_equal(host_u64(pts), ref["pts"])
    eps = U64_EPS if dtype == torch.float64 else F32_EPS
    tol_k = (1e-13 if dtype == torch.float64 else 1e-5) * kernel_scale(w)
    assert np.max(np.abs(k1.cpu().double().numpy() - ref["k1"])) <= tol_k
    tol_l = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel(lam.cpu().double().numpy(), ref["lam_ld"]) < tol_l
    # end to end: the GPU lambda carries its own rounding, so the solve bound
    # uses the oracle's spectrum and the dtype's unit roundoff
    tol_c = max(tol_l, solve_tol(ref["lam_ld"], w["sigma2"], y_host, ref["c_ld"], w["m"], eps))
    err_c = rel(c.cpu().double().numpy(), ref["c_ld"])
    assert err_c < tol_c, (err_c, tol_c)
    # log-det: each lambda_k has absolute error about eps * m * ||lambda|| / sqrt(n)
    lam_ld = ref["lam_ld"]
    n = lam_ld.shape[1]
    dl = 4 * eps * (w["m"] + 1) * np.linalg.norm(lam_ld, axis=1) / np.sqrt(n)
    tol_ld = dl * np.sum(1.0 / (lam_ld + w["sigma2"]), axis=1) + 1e-12 * np.abs(ref["logdet_ld"])
    assert np.all(np.abs(ld.cpu().numpy() - ref["logdet_ld"]) <= tol_ld)
    return err_c, tol_c


def test_workload1_net_order1(orc):
    w = W.workload(1)
    _check(orc, w, w["y"])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_workload2_lattice_full(orc, dtype):
    w = W.workload(2)
    x = W.to_unit_f64(orc.points(w))
    y = W.sine_response(x, w["eps"][:, 0, :])[:, None, :]
    _check(orc, w, np.ascontiguousarray(y), dtype)


def test_workload3_net_full_and_update(orc):
    w = W.workload(3)
    _check(orc, w, w["y"])
    # transform update 2^19 -> 2^20 equals the fresh transform
    n = 2 ** w["m"]
    y = torch.from_numpy(w["y"][:, 0, :]).cuda()
    yt_half = ldk.transform("dnet", y[:, : n // 2].contiguous())
    full = ldk.update_double("dnet", yt_half, y[:, n // 2:].contiguous())
    fresh = orc.transform("dnet", w["y"][:, 0, :], precise=True)
    assert rel(full.cpu().numpy(), fresh) < 1e-12
    # eigenvalue update: k1 of points [n/2, n) only
    ps, k = pointset(w), kernel(w)
    k1_lo = ldk.kernel_column(k, ps, 0, n // 2)
    k1_hi = ldk.kernel_column(k, ps, n // 2, n)
    lam_half = ldk.eig("dnet", k1_lo)
    lam_full = ldk.eig_update_double("dnet", lam_half, k1_hi)
    pts = orc.points(w)
    k1_ref = orc.kernel_column("dnet", pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"])
    assert rel(lam_full.cpu().numpy(), orc.eig("dnet", k1_ref, precise=True)) < 1e-12
