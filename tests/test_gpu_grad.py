"""GPU tests of the differentiable marginal likelihood
(``paper_2502_14256_amd.autograd``): ``.backward()`` against the oracle's
eigenbasis gradient (mll_grad), gated by ``ldk_dev.gate_vs_ld`` (10 times
the FP64 oracle's own error against its long-double twin, scaled by the unit
roundoff of the GPU's arithmetic; the stated 1e-12 / 1e-5 as floors), against central
differences of the FP64 GPU objective, at small sizes and at the gradient
workload's full size (net, n = 2^16, d = 64, 64 replications, order-2 DSI
kernel, FP32 and FP64 factors)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from paper_2502_14256_amd.autograd import marginal_log_likelihood
from ldk_dev import F32_EPS, U64_EPS, gate_vs_ld, pointset, record

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _theta(w):
    lg = torch.tensor(np.log(w["gamma"]), dtype=F64, device="cuda", requires_grad=True)
    lz = torch.tensor(math.log(w["zeta"]), dtype=F64, device="cuda", requires_grad=True)
    ls = torch.tensor(math.log(w["sigma2"]), dtype=F64, device="cuda", requires_grad=True)
    return lg, lz, ls


def _gpu(w, dtype, recompute=True, weights=None):
    lg, lz, ls = _theta(w)
    y = torch.from_numpy(np.ascontiguousarray(w["y"][:, 0, :])).cuda()
    L = marginal_log_likelihood(pointset(w), w["kind"], w["alpha"], lg, lz, ls, y, dtype=dtype,
                                recompute=recompute)
    wts = torch.ones_like(L) if weights is None else torch.as_tensor(weights, device="cuda")
    (L * wts).sum().backward()
    G = torch.cat([lg.grad, lz.grad.reshape(1), ls.grad.reshape(1)]).cpu().numpy()
    return L.detach().cpu().numpy(), G


def _check(name, w, ref, ref_ld, L, G, dtype):
    """Gate against the FP64 oracle: 10 times its own error (against the
    long-double twin) scaled by the unit roundoff of the GPU's factors and
    transform of y; floors 1e-12 (FP64) and 1e-5 (FP32) relative.  G is the
    gradient of sum_r L_r.  L is gated normwise over the replications (as G
    over its parameters): the oracle's error in one replication's L is a
    one-sample estimate of how the problem amplifies rounding, and it varies
    by 20x between the replications of one problem (5e-14 to 1e-12 relative
    on the lattice at n = 2^13, sigma^2 = 1e-3, where the GPU's L is within
    1.0-1.6e-12 in each)."""
    eps = U64_EPS if dtype == F64 else F32_EPS
    floor = 1e-12 if dtype == F64 else 1e-5
    Gref = ref["grad"].sum(axis=0)
    Gld = ref_ld["grad"].sum(axis=0)
    oL = gate_vs_ld(L, ref["L"], ref_ld["L"], eps, floor).max()
    oG = gate_vs_ld(G, Gref, Gld, eps, floor).max()
    rel_L = np.max(np.abs(L - ref["L"]) / np.abs(ref["L"]))
    rel_G = np.max(np.abs(G - Gref)) / np.max(np.abs(Gref))
    e_dd = np.max(np.abs(Gref - Gld)) / np.max(np.abs(Gld))
    record(name, L_over_gate=oL, grad_over_gate=oG, rel_L=rel_L, rel_grad=rel_G,
           oracle_rel_grad_vs_ld=e_dd)
    assert oL <= 1.0 and oG <= 1.0, (oL, oG, rel_L, rel_G, e_dd)


def _inst(kind, seed, m, d, R, sigma2=1e-3):
    w = W.small_lattice(seed, m, d, R) if kind == "lattice" else W.small_net(seed, m, d, R)
    w.update(alpha=np.full(d, 2, np.int32), gamma=1.0 / np.arange(1, d + 1) ** 2, zeta=1.2,
             sigma2=sigma2)
    return w


@pytest.mark.parametrize("kind,m,d", [("lattice", 13, 6), ("dnet", 13, 6), ("dnet", 10, 40),
                                      ("lattice", 8, 64), ("dnet", 8, 64)])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_backward_matches_oracle(orc, kind, m, d, dtype):
    w = _inst(kind, 90 + d, m, d, 3)
    ref, ref_ld = orc.mll_grad(w), orc.mll_grad_ld(w)
    L, G = _gpu(w, dtype)
    _check(f"autograd_{kind}_m{m}_d{d}_{'f64' if dtype == F64 else 'f32'}", w, ref, ref_ld, L, G,
           dtype)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_recompute_equals_stored(kind):
    w = _inst(kind, 5, 12, 5, 2)
    for dtype in (F64, F32):
        L1, G1 = _gpu(w, dtype, recompute=True)
        L2, G2 = _gpu(w, dtype, recompute=False)
        assert np.array_equal(L1, L2) and np.array_equal(G1, G2)


def test_backward_weights_replications(orc):
    # grad of sum_r c_r L_r is sum_r c_r grad L_r
    w = _inst("dnet", 17, 11, 4, 3)
    ref = orc.mll_grad(w)
    c = np.array([0.5, -2.0, 3.0])
    _, G = _gpu(w, F64, weights=c)
    want = (ref["grad"] * c[:, None]).sum(axis=0)
    assert np.max(np.abs(G - want)) <= 1e-9 * np.max(np.abs(want))


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_central_differences_fp64(orc, kind):
    """Central differences of the FP64 GPU objective (h = 1e-6, the step the
    gradient workload states).  Tolerance: the O(h^2) truncation, estimated
    from the same difference at 2h (Richardson: FD(2h) - FD(h) = 3 c h^2),
    plus the rounding of the two objective values over 2h.  That rounding
    is taken as 10 times the FP64 oracle's own error in L against its
    long-double twin (at least 8 (m + 4) u |L|): on lattices the small
    eigenvalues' rounding, amplified by |yt|^2 / (lambda + s2)^2, makes it
    about 1e-11 |L|, so h = 1e-6 resolves the derivative to about 1e-5."""
    m, d = 12, 4
    w = _inst(kind, 23, m, d, 1, sigma2=5e-3)
    e_dd_L = float(np.max(np.abs(orc.mll_grad(w)["L"] - orc.mll_grad_ld(w)["L"])))
    _, G = _gpu(w, F64)
    y = torch.from_numpy(np.ascontiguousarray(w["y"][:, 0, :])).cuda()
    th0 = np.concatenate([np.log(w["gamma"]), [math.log(w["zeta"]), math.log(w["sigma2"])]])

    def L(th):
        lg = torch.tensor(th[:d], dtype=F64, device="cuda")
        lz = torch.tensor(th[d], dtype=F64, device="cuda")
        ls = torch.tensor(th[d + 1], dtype=F64, device="cuda")
        return float(marginal_log_likelihood(pointset(w), kind, w["alpha"], lg, lz, ls, y,
                                             dtype=F64)[0])

    L0 = L(th0)
    dL = max(8 * (m + 4) * U64_EPS * abs(L0), 10 * e_dd_L)
    for h in (1e-6,):
        for p in range(d + 2):
            e = np.zeros(d + 2)
            e[p] = h
            fd1 = (L(th0 + e) - L(th0 - e)) / (2 * h)
            fd2 = (L(th0 + 2 * e) - L(th0 - 2 * e)) / (4 * h)
            trunc = abs(fd2 - fd1) / 3.0
            tol = 2 * trunc + 2 * 2 * dL / (2 * h) + 2 * dL / (4 * h)
            record(f"fd_{kind}_p{p}", err=abs(fd1 - G[p]), tol=tol)
            assert abs(fd1 - G[p]) <= tol, (p, fd1, G[p], tol)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gradient_workload_full_size(orc, dtype):
    """The gradient workload at its full size: LMS + digitally shifted net,
    n = 2^16, d = 64, 64 replications, order-2 DSI kernel, gamma_j = 1/j^2,
    sigma2 = 1e-3 (FP32 and FP64 factors) against the oracle."""
    w = W.workload(5)
    ref, ref_ld = orc.mll_grad(w), orc.mll_grad_ld(w)
    L, G = _gpu(w, dtype)
    _check(f"autograd_workload5_{'f64' if dtype == F64 else 'f32'}", w, ref, ref_ld, L, G, dtype)
    # FP32 against FP64 on the GPU, stated per result
    if dtype == F32:
        L64, G64 = _gpu(w, F64)
        record("autograd_workload5_f32_vs_f64",
               rel_L=float(np.max(np.abs(L - L64) / np.abs(L64))),
               rel_grad=float(np.max(np.abs(G - G64)) / np.max(np.abs(G64))))
