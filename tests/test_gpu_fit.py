"""ldk_fit (eigenvalues, solves and log-det in one call) against the separate
entry points: the same eigenvalues and solutions bit for bit (the fused path
runs the same tile arithmetic, reading the eigenvalues back from its own
writes), the log-det to rounding (another fixed summation order)."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import kernel, pointset

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 2, 3, 6, 12, 13, 16, 20])
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
    assert torch.equal(lam, lam_ref)
    if nrhs:
        c_ref = ldk.solve(kind, lam_ref, s2, y)
        assert torch.equal(c, c_ref)
    ld_ref = ldk.logdet(lam_ref, s2)
    assert torch.allclose(ld, ld_ref, rtol=1e-13, atol=1e-13 * n, equal_nan=True)
