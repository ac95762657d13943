"""GPU parity of the marginal-likelihood path against the oracle: the
likelihood and dL/dlambda, the adjoint back to dL/dk1, the kernel-parameter
gradient, and the whole gradient step (points -> k1 -> lambda -> L, g ->
dL/dk1 -> gradient)."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import kernel, kernel_scale, pointset, record, rel

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _inst(kind, seed, m, d, R, alpha, gamma, zeta=1.0, sigma2=1e-3):
    w = W.small_lattice(seed, m, d, R) if kind == "lattice" else W.small_net(seed, m, d, R)
    w.update(alpha=np.array(alpha, np.int32), gamma=np.array(gamma, np.float64), zeta=zeta,
             sigma2=sigma2)
    return w


def _lam(orc, w):
    pts = orc.points(w)
    k1 = orc.kernel_column(w["kind"], pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"])
    return k1, orc.eig(w["kind"], k1)[0]


MLL_M = [0, 1, 2, 3, 5, 11, 12, 13, 14, 16, 20]


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", MLL_M)
@pytest.mark.parametrize("dtype", [F64, F32])
def test_mll_likelihood_and_dlambda(orc, kind, m, dtype):
    R = 2 if m < 16 else 1
    alpha = [2, 1, 3] if kind == "lattice" else [2, 4, 1]
    w = _inst(kind, 40 + m, m, 3, R, alpha, [0.9, 0.5, 0.3], sigma2=1e-2)
    _, lam = _lam(orc, w)
    y = w["y"][:, 0, :].astype(np.float64 if dtype == F64 else np.float32)
    L_ref, g_ref, ds_ref = orc.mll(kind, lam, w["sigma2"], y.astype(np.float64))
    L, g, ds = ldk.mll(kind, torch.from_numpy(lam).cuda(), w["sigma2"], torch.from_numpy(y).cuda())
    L, g, ds = L.cpu().numpy(), g.cpu().numpy(), ds.cpu().numpy()
    # FP32 rows: |yt|^2 carries the float transform's rounding (~m eps32)
    tol = 1e-12 if dtype == F64 else 4e-6 * max(m, 1)
    eL = np.max(np.abs(L - L_ref) / np.maximum(1.0, np.abs(L_ref)))
    eg = rel(g, g_ref)
    eds = np.max(np.abs(ds - ds_ref) / np.maximum(1.0, np.abs(ds_ref)))
    record(f"mll_{kind}_m{m}_{'f64' if dtype == F64 else 'f32'}", err_L=eL, err_g=eg, err_ds=eds,
           tol=tol)
    assert eL < tol and eg < tol and eds < tol, (eL, eg, eds, tol)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 2, 3, 6, 12, 13, 14, 19, 21])
def test_mll_adjoint(orc, kind, m):
    rng = np.random.default_rng(500 + m)
    R = 3 if m < 19 else 1
    g = rng.standard_normal((R, 2**m))  # no symmetry: the real part is what is defined
    a_ref = orc.mll_adjoint(kind, g)
    gd = torch.from_numpy(g).cuda()
    a = ldk.mll_adjoint(kind, gd).cpu().numpy()
    err = rel(a, a_ref)
    record(f"mll_adjoint_{kind}_m{m}", err=err)
    assert err < 1e-13 * max(m, 1), err
    # exact aliasing: a written over g
    ldk.mll_adjoint(kind, gd, out=gd)
    assert np.array_equal(gd.cpu().numpy(), a)


def _grad_case(kind, uniform, seed=7, m=12, d=5, R=2):
    if kind == "lattice":
        alpha = [2] * d if uniform else [1, 2, 3, 2, 1][:d]
    else:
        alpha = [2] * d if uniform else [1, 2, 3, 4, 2][:d]
    return _inst(kind, seed, m, d, R, alpha, 0.8 ** np.arange(1, d + 1), zeta=1.3)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("src", ["regen", "pts"])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("window", [(0, 4096), (100, 3001)])
@pytest.mark.parametrize("with_k1", [False, True])
def test_kernel_grad(orc, kind, uniform, src, dtype, window, with_k1):
    w = _grad_case(kind, uniform)
    n_min, n_max = window
    pts_all = orc.points(w, 0, n_max)
    x0 = pts_all[:, 0, :]
    pts = pts_all[:, n_min:, :]
    rng = np.random.default_rng(9)
    a = rng.standard_normal((w["R"], n_max - n_min))
    ref = orc.kernel_grad(kind, pts, x0, w["alpha"], w["gamma"], w["zeta"], a)
    ps, k = pointset(w), kernel(w)
    ad = torch.from_numpy(a).cuda()
    if src == "regen":
        k1 = ldk.kernel_column(k, ps, n_min, n_max, dtype=dtype) if with_k1 else None
        got = ldk.kernel_grad(k, ps, n_min, n_max, ad, dtype=dtype, k1=k1)
    else:
        from ldk_dev import dev_u64
        pd, xd = dev_u64(pts), dev_u64(x0)
        k1 = (ldk.kernel_column(k, ps, n_min, n_max, pts=pd, x0=xd, dtype=dtype) if with_k1
              else None)
        got = ldk.kernel_grad(k, ps, n_min, n_max, ad, pts=pd, x0=xd, dtype=dtype, k1=k1)
    got = got.cpu().numpy()
    # |d k1_i / d theta| <= the kernel scale, so each sum is off by at most
    # tol * ||a||_1 * scale
    bound = np.abs(a).sum(axis=1, keepdims=True) * kernel_scale(w)
    tol = 1e-14 if dtype == F64 else 2e-6
    err = np.max(np.abs(got - ref) / bound)
    record(f"kernel_grad_{kind}_{'u' if uniform else 'mix'}_{src}_{window}_{dtype}"
           f"{'_k1' if with_k1 else ''}", err=err, tol=tol)
    assert err < tol, (err, got, ref)


def test_kernel_grad_exactly_zero_factor(orc):
    """DSI order 1 with gamma = 2: the factor is 0 on [1/2, 1); the product of
    the other factors must not come from a division by it."""
    w = _inst("dnet", 13, 10, 3, 1, [1, 2, 1], [2.0, 0.5, 2.0])
    pts = orc.points(w)
    a = np.random.default_rng(3).standard_normal((1, 2**10))
    ref = orc.kernel_grad("dnet", pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"], a)
    for dtype, with_k1 in ((F64, False), (F32, False), (F64, True), (F32, True)):
        k1 = (ldk.kernel_column(kernel(w), pointset(w), 0, 2**10, dtype=dtype) if with_k1
              else None)
        if with_k1:
            # zeros in k1: those tiles must take the two sweeps
            assert torch.any(k1 == 0)
        got = ldk.kernel_grad(kernel(w), pointset(w), 0, 2**10, torch.from_numpy(a).cuda(),
                              dtype=dtype, k1=k1).cpu().numpy()
        assert np.all(np.isfinite(got))
        bound = np.abs(a).sum() * kernel_scale(w)
        assert np.max(np.abs(got - ref)) / bound < (1e-14 if dtype == F64 else 2e-6)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_kernel_grad_empty_window(kind):
    w = _grad_case(kind, True)
    out = torch.full((w["R"], w["d"] + 1), 7.0, dtype=F64, device="cuda")
    ldk.kernel_grad(kernel(w), pointset(w), 64, 64, torch.empty((w["R"], 0), dtype=F64,
                                                                device="cuda"), out=out)
    assert torch.all(out == 0)


@pytest.mark.parametrize("kind,m,d", [("lattice", 13, 6), ("dnet", 13, 6), ("dnet", 10, 40)])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gradient_step_end_to_end(orc, kind, m, d, dtype):
    """The whole gradient step on the GPU against the oracle's mll_grad (FP64
    throughout).  FP32 runs the kernel, its transforms and the transform of y
    in float (eigenvalues, g, adjoint and sums stay FP64): its error is
    recorded against the FP64 oracle."""
    R = 3
    alpha = [2] * d
    w = _inst(kind, 70 + d, m, d, R, alpha, 1.0 / np.arange(1, d + 1) ** 2, sigma2=1e-3)
    ref = orc.mll_grad(w)
    n = 2**m
    ps, k = pointset(w), kernel(w)
    k1 = ldk.kernel_column(k, ps, 0, n, dtype=dtype)
    lam = ldk.eig(kind, k1)
    y = torch.from_numpy(w["y"][:, 0, :]).cuda().to(dtype)
    L, g, ds = ldk.mll(kind, lam, w["sigma2"], y)
    a = ldk.mll_adjoint(kind, g)
    kg = ldk.kernel_grad(k, ps, 0, n, a, dtype=dtype)
    kg1 = ldk.kernel_grad(k, ps, 0, n, a, dtype=dtype, k1=k1)
    grad = torch.cat([kg, ds[:, None]], dim=1).cpu().numpy()
    grad1 = torch.cat([kg1, ds[:, None]], dim=1).cpu().numpy()
    Lh = L.cpu().numpy()
    eL = np.max(np.abs(Lh - ref["L"]) / np.abs(ref["L"]))
    eG = max(np.max(np.abs(gr - ref["grad"])) / np.max(np.abs(ref["grad"]))
             for gr in (grad, grad1))
    # gate: 10x the FP64 oracle's own error against its long-double twin,
    # scaled by the unit roundoff of the GPU's factors (ldk_dev.gate_vs_ld);
    # L normwise over the replications, as every other result is over its
    # vector: the oracle's error in one replication's L is a one-sample
    # estimate of how the problem amplifies rounding, and it varies by 20x
    # between replications of one problem (5e-14 to 1e-12 relative on the
    # lattice at n = 2^13, sigma^2 = 1e-3)
    from ldk_dev import F32_EPS, U64_EPS, gate_vs_ld
    ref_ld = orc.mll_grad_ld(w)
    eps = U64_EPS if dtype == F64 else F32_EPS
    floor = 1e-12 if dtype == F64 else 1e-5
    oL = gate_vs_ld(Lh, ref["L"], ref_ld["L"], eps, floor).max()
    oG = max(gate_vs_ld(gr, ref["grad"], ref_ld["grad"], eps, floor).max() for gr in (grad, grad1))
    record(f"grad_step_{kind}_m{m}_d{d}_{'f64' if dtype == F64 else 'f32'}", err_L=eL, err_grad=eG,
           L_over_gate=oL, grad_over_gate=oG)
    assert oL <= 1.0 and oG <= 1.0, (oL, oG, eL, eG)
