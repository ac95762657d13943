"""ldk_fit (eigenvalues, solves and log-det in one call) against the separate
entry points, to rounding: the fused FP64 lattice path runs the same
transform arithmetic, but with one right-hand side both top passes share one
kernel whose instruction schedule (and so the rounding of a fused
multiply-add here and there) differs; the log-det sums in another fixed
order.  Bounds: the eigenvalues within the transform's normwise rounding
bound; the solutions within twice the solve's first-order rounding bound
(as solve_tol, with max 1/|lambda + s2|) plus twice the first-order effect of the measured eigenvalue
difference, |dc| <= max_k |dlambda_k| / (lambda_k + s2)^2 |y| (each side
filters with its own eigenvalues)."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import kernel, pointset

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 2, 3, 6, 9, 10, 11, 12, 13, 16, 17, 20, 21])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nrhs", [0, 1, 3])
def test_fit_equals_separate_calls(kind, m, dtype, nrhs):
    if m >= 16 and nrhs == 3:
        nrhs = 2
    R = 2 if m < 16 else 1
    d = 5
    w = (W.small_lattice if kind == "lattice" else W.small_net)(70 + m, m, d, R, nrhs=max(nrhs, 1))
    w.update(alpha=np.full(d, 2, np.int32), gamma=0.7 ** np.arange(1, d + 1), zeta=1.0)
    n = 2**m
    k1 = ldk.kernel_column(kernel(w), pointset(w), 0, n, dtype=dtype)
    y = torch.from_numpy(w["y"][:, :nrhs]).cuda().to(dtype).contiguous()
    s2 = 1e-3
    lam, c, ld = ldk.fit(kind, k1, s2, y)
    lam_ref = ldk.eig(kind, k1)
    eps = float(np.finfo(np.float64 if dtype == torch.float64 else np.float32).eps)
    dl = (lam - lam_ref).abs().max().item()
    assert dl <= 8 * (m + 1) * eps * lam_ref.abs().max().item(), dl
    if nrhs:
        c_ref = ldk.solve(kind, lam_ref, s2, y)
        cr, cg = c_ref.double().cpu().numpy(), c.double().cpu().numpy()
        yr = y.double().cpu().numpy().reshape(R, -1)
        lr, lg = lam_ref.cpu().numpy(), lam.cpu().numpy()
        for r in range(R):
            cn = max(np.linalg.norm(cr[r]), 1e-300)
            # solve_tol's bound with max 1/|lambda + s2| (FP32 columns can
            # give slightly negative eigenvalues)
            tol = 2 * 4.0 * (2 * m + 2) * eps * np.max(1 / np.abs(lr[r] + s2)) * \
                np.linalg.norm(yr[r]) / cn
            pert = np.max(np.abs(lg[r] - lr[r]) / (lr[r] + s2) ** 2) * np.linalg.norm(yr[r]) / cn
            err = np.linalg.norm(cg[r] - cr[r]) / cn
            assert err <= tol + 2 * pert, (r, err, tol, pert)
    ld_ref = ldk.logdet(lam_ref, s2)
    assert torch.allclose(ld, ld_ref, rtol=1e-13, atol=1e-13 * n, equal_nan=True)


@pytest.mark.parametrize("kind,dtype", [("dnet", torch.float64), ("lattice", torch.float32),
                                        ("lattice", torch.float64)])
@pytest.mark.parametrize("m", [4, 10, 12, 16])
def test_fit_without_logdet(kind, dtype, m):
    # no log-det output (a NULL pointer): the one-launch net fit and the
    # FP32 lattice fit that carries log-det partials must give the same
    # eigenvalues and solutions bit for bit as with it
    R, d, nrhs = 2, 5, 2
    w = (W.small_lattice if kind == "lattice" else W.small_net)(90 + m, m, d, R, nrhs=nrhs)
    w.update(alpha=np.full(d, 2, np.int32), gamma=0.7 ** np.arange(1, d + 1), zeta=1.0)
    k1 = ldk.kernel_column(kernel(w), pointset(w), 0, 2**m, dtype=dtype)
    y = torch.from_numpy(w["y"][:, :nrhs]).cuda().to(dtype).contiguous()
    lam, c, ld = ldk.fit(kind, k1, 1e-3, y)
    lam0, c0, ld0 = ldk.fit(kind, k1, 1e-3, y, logdet=False)
    assert ld0 is None and ld is not None
    assert torch.equal(lam0, lam) and torch.equal(c0, c)
