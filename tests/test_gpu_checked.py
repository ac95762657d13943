"""GPU tests of the checked entry points (ldk_solve_checked,
ldk_logdet_checked: K + sigma^2 I = V (Lambda + sigma^2 I) conj(V) is
positive definite exactly when every lambda_k + sigma^2 > 0, Sec. 5.4) and
of the binding's refusal of undersized or misplaced buffers (raised on the
host, before any device call)."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import kernel, pointset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _init():
    ldk.init()


def _fit_inputs(kind, m=12, d=4, R=3, nrhs=2):
    w = W.small_net(41, m, d, R, nrhs=nrhs) if kind == "dnet" else \
        W.small_lattice(41, m, d, R, nrhs=nrhs)
    w.update(alpha=np.full(d, 2, np.int32), gamma=1.0 / np.arange(1, d + 1) ** 2, zeta=1.0)
    ps, k = pointset(w), kernel(w)
    k1 = ldk.kernel_column(k, ps, 0, 2**m)
    lam = ldk.eig(kind, k1)
    y = torch.from_numpy(np.asarray(w["y"], np.float64).reshape(R, nrhs, 2**m)).cuda()
    return lam, y


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_checked_equals_plain_when_spd(kind):
    lam, y = _fit_inputs(kind)
    s2 = 1e-3
    c0 = ldk.solve(kind, lam, s2, y)
    c1 = ldk.solve(kind, lam, s2, y, checked=True)
    l0 = ldk.logdet(lam, s2)
    l1 = ldk.logdet(lam, s2, checked=True)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1) and torch.equal(l0, l1)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("bad", ["negative", "nan", "zero_sum"])
def test_checked_reports_not_spd(kind, bad):
    lam, y = _fit_inputs(kind)
    s2 = 1e-3
    lam = lam.clone()
    r, k = 1, 77
    if bad == "negative":
        lam[r, k] = -1.0
    elif bad == "nan":
        lam[r, k] = float("nan")
    else:
        lam[r, k] = -s2  # lambda + sigma^2 == 0 exactly
    c = torch.full_like(y, 7.0)
    with pytest.raises(ldk.LdkError, match=r"status -4"):
        ldk.solve(kind, lam, s2, y, out=c, checked=True)
    out = torch.full((lam.shape[0],), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ldk.LdkError, match=r"status -4"):
        ldk.logdet(lam, s2, out=out, checked=True)
    torch.cuda.synchronize()
    # nothing was enqueued: the outputs keep their contents
    assert bool((c == 7.0).all()) and bool((out == 7.0).all())
    # the unchecked log-det gives NaN for exactly the bad row
    ld = ldk.logdet(lam, s2).cpu().numpy()
    assert np.isnan(ld[r]) and np.all(np.isfinite(np.delete(ld, r)))


def test_checked_calls_repeat_cleanly():
    # the device counter is cleared by every checked call
    lam, y = _fit_inputs("dnet")
    bad = lam.clone()
    bad[0, 0] = -5.0
    for _ in range(3):
        with pytest.raises(ldk.LdkError):
            ldk.logdet(bad, 0.0, checked=True)
        ldk.logdet(lam, 1e-3, checked=True)


def test_binding_rejects_undersized_buffers():
    lam, y = _fit_inputs("dnet", m=10, R=2, nrhs=3)
    R, nrhs, n = y.shape
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.solve("dnet", lam, 1e-3, y, out=torch.empty(R * nrhs * n - 1, dtype=torch.float64,
                                                       device="cuda"))
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.solve("dnet", lam[:1], 1e-3, y)  # lambda rows for R replications
    with pytest.raises(ldk.LdkError, match="bytes"):
        ldk.fit("lattice", torch.zeros((R, n), dtype=torch.float64, device="cuda"), 1e-3, y,
                ws=torch.empty(16, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ldk.LdkError, match="float64"):
        ldk.logdet(lam, 1e-3, out=torch.empty(R, dtype=torch.float32, device="cuda"))
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.eig("dnet", lam, out=torch.empty((R, n // 2), dtype=torch.float64, device="cuda"))
    with pytest.raises(ldk.LdkError):
        ldk.solve("dnet", lam, 1e-3, y, out=torch.empty_like(y, device="cpu"))
    w = W.small_net(3, 8, 5, 4)
    ps = pointset(w)
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.gen_points(ps, 0, 256, out=torch.empty((4, 255, 5), dtype=torch.int64, device="cuda"))
    coef = torch.ones(5, dtype=torch.float64, device="cuda")
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.rqmc(ps, 256, "corner_peak", coef,
                 mu_r=torch.empty(3, dtype=torch.float64, device="cuda"))
    with pytest.raises(ldk.LdkError, match="bytes"):
        ldk.rqmc(ps, 256, "corner_peak", coef, ws=torch.empty(8, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ldk.LdkError, match="elements"):
        ldk.rqmc(ps, 256, "corner_peak", torch.ones(4, dtype=torch.float64, device="cuda"))
