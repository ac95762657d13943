"""Split-FP16 matrix-core Walsh-Hadamard transform against the oracle's FP64
FWHT: normwise error within the FP32 transform tolerance, over sizes that
exercise the per-row kernel (m < 12, leftover of 1-3 index bits), the
register-resident passes (m >= 12: one row pass, one column pass of 1-8
bits, two column passes), rows not 16-byte aligned, and data spanning a
wide dynamic range (the per-stage power-of-two scaling).  Then the FP32
digital-net solve and matvec on the matrix-core passes (tuned-table engine
1) against the oracle with the FP32 solve gate."""
import numpy as np
import pytest
import torch

import paper_2502_14256_amd as ldk
from ldk_dev import record, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5, 7, 8, 11, 12, 13, 14, 15, 16, 17, 19, 20, 21, 22])
def test_fwht_split16_matches_oracle(orc, m):
    rng = np.random.default_rng(600 + m)
    B = 3 if m < 18 else 1
    x = (rng.standard_normal((B, 2**m)) * np.exp(rng.uniform(-8, 8, (B, 2**m)))).astype(np.float32)
    ref = orc.transform("dnet", x.astype(np.float64), precise=True)
    xd = torch.from_numpy(x).cuda()
    y = ldk.fwht_split16(xd).cpu().numpy()
    err = rel(y, ref)
    # the FP32 butterfly transform on the same data, for comparison
    e32 = rel(ldk.transform("dnet", xd).cpu().numpy(), ref)
    record(f"fwht_split16_m{m}", err=err, err_fp32_butterflies=e32)
    assert err < 2e-6, (err, e32)
    # in place
    ldk.fwht_split16(xd, out=xd)
    assert np.array_equal(xd.cpu().numpy(), y)


def test_fwht_split16_zero_and_tiny_rows():
    x = torch.zeros((2, 2**12), dtype=torch.float32, device="cuda")
    x[1, 5] = 1e-30  # far below the FP16 range: scaled up before the split
    y = ldk.fwht_split16(x).cpu().numpy()
    assert np.all(y[0] == 0)
    assert np.allclose(y[1], 1e-30 / 64 * np.where(np.array([bin(k & 5).count("1") % 2 for k in range(4096)]) == 1, -1, 1), rtol=1e-6, atol=0)


@pytest.mark.parametrize("m", [12, 16, 21])
def test_fwht_split16_unaligned_rows(orc, m):
    # rows starting 4 bytes past a 16-byte boundary take the scalar loads
    rng = np.random.default_rng(650 + m)
    B, n = 2, 2**m
    x = rng.standard_normal((B, n)).astype(np.float32)
    buf = torch.zeros(B * n + 1, dtype=torch.float32, device="cuda")
    xd = buf[1:].view(B, n)
    xd.copy_(torch.from_numpy(x))
    assert xd.data_ptr() % 16 == 4
    ref = orc.transform("dnet", x.astype(np.float64), precise=True)
    out = torch.zeros(B * n + 1, dtype=torch.float32, device="cuda")[1:].view(B, n)
    y = ldk.fwht_split16(xd, out=out).cpu().numpy()
    assert rel(y, ref) < 2e-6
    # the aligned call gives the same bits (same arithmetic, other loads)
    assert np.array_equal(ldk.fwht_split16(torch.from_numpy(x).cuda()).cpu().numpy(), y)


@pytest.fixture
def split16_table(tmp_path):
    """A tuned table selecting the matrix-core passes for FP32 net solves at
    every m >= 12 and every row count."""
    ldk.init()
    p = tmp_path / "split16.txt"
    p.write_text("".join(f"{ldk.DNET_B2} {ldk.F32} {m} 0 12 3 1\n" for m in range(12, 27)))
    ldk.load_tuned(str(p))
    yield
    ldk.load_tuned(None)


@pytest.mark.parametrize("m,R,nrhs", [(12, 1, 1), (13, 2, 3), (16, 1, 4), (20, 1, 2), (21, 1, 1)])
def test_split16_solve_and_matvec_match_oracle(orc, split16_table, m, R, nrhs):
    import workloads as W
    from ldk_dev import F32_EPS, kernel, pointset, solve_tol
    assert ldk.plan_info("dnet", ldk.F32, m, R * nrhs)["engine"] == 1
    w = W.small_net(41 + m, m, 5, R, nrhs=nrhs)
    w.update(alpha=np.full(5, 2, np.int32), gamma=1.0 / np.arange(1, 6) ** 2, zeta=1.0,
             sigma2=1e-3)
    n = 2**m
    k1 = ldk.kernel_column(kernel(w), pointset(w), 0, n, dtype=torch.float32)
    lam_ref = orc.eig("dnet", k1.cpu().double().numpy(), precise=True)
    lam = ldk.eig("dnet", k1)  # FP64 eigenvalues of the FP32 column
    y = torch.from_numpy(w["y"]).float().cuda()
    yh = y.cpu().double().numpy()
    c_ref = orc.solve("dnet", lam_ref, w["sigma2"], yh, precise=True)
    c = ldk.solve("dnet", lam, w["sigma2"], y).cpu().double().numpy()
    v = ldk.matvec("dnet", lam, y).cpu().double().numpy()
    # the split costs at most one FP16 rounding of the low term (2^-22 of
    # the scaled element) per radix-16 stage on top of the FP32 sums: twice
    # the per-level rounding of the butterflies
    tol = max(1e-5, 2 * solve_tol(lam_ref, w["sigma2"], yh, c_ref, m, F32_EPS))
    err = rel(c, c_ref)
    # matvec K y: the same first-order bound with D = diag(lambda)
    v_ref = orc.matvec("dnet", lam_ref, yh, precise=True)
    ratio = np.max(np.abs(lam_ref)) * np.linalg.norm(yh) / np.linalg.norm(v_ref)
    tol_v = max(1e-5, 2 * 4.0 * (2 * m + 2) * F32_EPS * ratio)
    err_v = rel(v, v_ref)
    # the butterfly engine on the same inputs, for the record
    ldk.load_tuned(None)
    c_b = ldk.solve("dnet", lam, w["sigma2"], y).cpu().double().numpy()
    v_b = ldk.matvec("dnet", lam, y).cpu().double().numpy()
    record(f"split16_solve_m{m}_R{R}_nrhs{nrhs}", err=err, err_butterflies=rel(c_b, c_ref),
           tol=tol, err_matvec=err_v, err_matvec_butterflies=rel(v_b, v_ref), tol_matvec=tol_v)
    assert err < tol, (err, tol, rel(c_b, c_ref))
    assert err_v < tol_v, (err_v, tol_v, rel(v_b, v_ref))


@pytest.mark.parametrize("m", [12, 13, 16, 20])
def test_split16_likelihood_matches_oracle(orc, split16_table, m):
    # the likelihood's |H y|^2 for FP32 net rows on the matrix-core passes:
    # the FP32 gate of the butterfly path
    import workloads as W
    R = 2 if m < 16 else 1
    w = W.small_net(40 + m, m, 3, R)
    w.update(alpha=np.array([2, 4, 1], np.int32), gamma=np.array([0.9, 0.5, 0.3]), zeta=1.0,
             sigma2=1e-2)
    assert ldk.plan_info("dnet", ldk.F32, m, R)["engine"] == 1
    pts = orc.points(w)
    k1 = orc.kernel_column("dnet", pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"])
    lam = orc.eig("dnet", k1)[0]
    y = w["y"][:, 0, :].astype(np.float32)
    L_ref, g_ref, ds_ref = orc.mll("dnet", lam, w["sigma2"], y.astype(np.float64))
    L, g, ds = (t.cpu().numpy() for t in ldk.mll("dnet", torch.from_numpy(lam).cuda(), w["sigma2"],
                                                  torch.from_numpy(y).cuda()))
    tol = 4e-6 * m
    eL = np.max(np.abs(L - L_ref) / np.maximum(1.0, np.abs(L_ref)))
    eg = rel(g, g_ref)
    eds = np.max(np.abs(ds - ds_ref) / np.maximum(1.0, np.abs(ds_ref)))
    record(f"split16_mll_dnet_m{m}", err_L=eL, err_g=eg, err_ds=eds, tol=tol)
    assert eL < tol and eg < tol and eds < tol, (eL, eg, eds, tol)


def test_split16_gradient_step_matches_oracle(orc, split16_table):
    # the FP32 gradient step with the matrix-core transform of y, gated like
    # the butterfly path (10x the FP64 oracle's own error, FP32 unit roundoff)
    import workloads as W
    from ldk_dev import F32_EPS, gate_vs_ld, kernel, pointset
    m, d, R = 13, 6, 3
    w = W.small_net(76, m, d, R)
    w.update(alpha=np.full(d, 2, np.int32), gamma=1.0 / np.arange(1, d + 1) ** 2, zeta=1.0,
             sigma2=1e-3)
    ref, ref_ld = orc.mll_grad(w), orc.mll_grad_ld(w)
    n = 2**m
    ps, k = pointset(w), kernel(w)
    k1 = ldk.kernel_column(k, ps, 0, n, dtype=torch.float32)
    lam = ldk.eig("dnet", k1)
    y = torch.from_numpy(w["y"][:, 0, :]).cuda().float()
    L, g, ds = ldk.mll("dnet", lam, w["sigma2"], y)
    kg = ldk.kernel_grad(k, ps, 0, n, ldk.mll_adjoint("dnet", g), dtype=torch.float32, k1=k1)
    grad = torch.cat([kg, ds[:, None]], dim=1).cpu().numpy()
    Lh = L.cpu().numpy()
    oL = gate_vs_ld(Lh[:, None], ref["L"][:, None], ref_ld["L"][:, None], F32_EPS, 1e-5).max()
    oG = gate_vs_ld(grad, ref["grad"], ref_ld["grad"], F32_EPS, 1e-5).max()
    record("split16_grad_step_dnet_m13_d6", L_over_gate=oL, grad_over_gate=oG)
    assert oL <= 1.0 and oG <= 1.0, (oL, oG)


@pytest.mark.parametrize("m", [12, 16])
def test_split16_solve_unaligned_rows(split16_table, m):
    # rows 4 bytes past a 16-byte boundary: the row passes load and store
    # element by element; same arithmetic, so the same bits as aligned rows
    rng = np.random.default_rng(70 + m)
    R, nrhs, n = 2, 3, 2**m
    lam = torch.from_numpy(1.0 + rng.random((R, n))).cuda()
    y = torch.from_numpy(rng.standard_normal((R, nrhs, n))).float().cuda()
    want = ldk.solve("dnet", lam, 1e-3, y)
    yb = torch.zeros(R * nrhs * n + 1, dtype=torch.float32, device="cuda")[1:].view(R, nrhs, n)
    cb = torch.zeros(R * nrhs * n + 1, dtype=torch.float32, device="cuda")[1:].view(R, nrhs, n)
    yb.copy_(y)
    assert yb.data_ptr() % 16 == 4 and cb.data_ptr() % 16 == 4
    got = ldk.solve("dnet", lam, 1e-3, yb, out=cb)
    assert torch.equal(got, want)
