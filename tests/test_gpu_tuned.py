"""GPU tests of the tuned transform plans (ldk_init_tuned): eigenvalues,
solves and the fused fit under every candidate plan the tuner may choose
(tile 2^9 .. 2^12, radix 4 or 8) against the oracle with the same gates as
the default plan; the table's loading rules; and the tuner itself on a tiny
case list."""
import os

import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import F32_EPS, U64_EPS, kernel, pointset, rel, solve_tol

pytestmark = pytest.mark.gpu

KIND_CODE = {"lattice": 0, "dnet": 1}


@pytest.fixture(autouse=True)
def _default_table():
    ldk.init()
    yield
    ldk.load_tuned(None)


def _load(tmp_path, lines):
    p = tmp_path / "table.txt"
    p.write_text("".join(lines))
    ldk.load_tuned(str(p))


def _line(kind, dt, m, rows, lt, lr):
    return f"{KIND_CODE[kind]} {dt} {m} {int(np.log2(rows))} {lt} {lr}\n"


@pytest.mark.parametrize("kind,m,dtype", [("lattice", 13, torch.float64), ("dnet", 14, torch.float64),
                                          ("lattice", 16, torch.float32), ("dnet", 16, torch.float32),
                                          ("lattice", 20, torch.float64)])
def test_solve_and_eig_under_every_candidate_plan(orc, tmp_path, kind, m, dtype):
    R, nrhs = 1, 3
    w = W.small_net(31, m, 5, R, nrhs=nrhs) if kind == "dnet" else \
        W.small_lattice(31, m, 5, R, nrhs=nrhs)
    w.update(alpha=np.full(5, 2, np.int32), gamma=1.0 / np.arange(1, 6) ** 2, zeta=1.0,
             sigma2=1e-3)
    n = 2 ** m
    dt = ldk.F64 if dtype == torch.float64 else ldk.F32
    k1 = ldk.kernel_column(kernel(w), pointset(w), 0, n, dtype=dtype)
    k1h = k1.cpu().double().numpy()
    lam_ref = orc.eig(kind, k1h, precise=True)
    y = torch.from_numpy(w["y"]).to(dtype).cuda()
    yh = y.cpu().double().numpy()
    c_ref = orc.solve(kind, lam_ref, w["sigma2"], yh, precise=True)
    eps = U64_EPS if dtype == torch.float64 else F32_EPS
    tried = 0
    for lt in (9, 10, 11, 12):
        for lr in (2, 3):
            try:
                _load(tmp_path, [_line(kind, dt, m, nrhs, lt, lr), _line(kind, ldk.F64, m, 1, lt, lr)])
            except ldk.LdkError:
                continue  # a plan the pass kernels cannot run
            info = ldk.plan_info(kind, dt, m, nrhs)
            assert info["log_tile"] == lt and info["radix"] == 2 ** lr
            tried += 1
            lam = ldk.eig(kind, k1)
            err_l = rel(lam.cpu().numpy(), lam_ref)
            assert err_l < 1e-12, (lt, lr, err_l)  # FP64 transform either way
            c = ldk.solve(kind, lam, w["sigma2"], y)
            err_c = rel(c.cpu().double().numpy(), c_ref)
            tol = max(1e-12 if dtype == torch.float64 else 1e-5,
                      solve_tol(lam_ref, w["sigma2"], yh, c_ref, m, eps),
                      # the GPU's own eigenvalues: their normwise error enters
                      # the solve through 1/(lambda + s2)
                      4 * err_l * np.max(np.abs(lam_ref)) / (np.min(lam_ref) + w["sigma2"]))
            assert err_c < tol, (lt, lr, err_c, tol)
    assert tried >= 3


def test_fused_fit_under_tuned_plans(orc, tmp_path):
    # the FP64 lattice fit shares its passes between the column and the
    # responses: every candidate against the oracle end to end
    w = W.workload(2)
    m = w["m"]
    x = W.to_unit_f64(orc.points(w))
    y = np.ascontiguousarray(W.sine_response(x, w["eps"][:, 0, :])[:, None, :])
    ref = orc.fit_solve(w, y=y, precise=True)
    e64 = rel(ref["c"], ref["c_ld"])
    ps, k = pointset(w), kernel(w)
    k1 = ldk.kernel_column(k, ps, 0, 2 ** m)
    yd = torch.from_numpy(y).cuda()
    for lt in (10, 11, 12):
        for lr in (2, 3):
            try:
                _load(tmp_path, [_line("lattice", ldk.F64, m, 2, lt, lr)])
            except ldk.LdkError:
                continue
            lam, c, ld = ldk.fit("lattice", k1, w["sigma2"], yd)
            assert rel(lam.cpu().numpy(), ref["lam_ld"]) < 1e-12, (lt, lr)
            err = rel(c.cpu().numpy(), ref["c_ld"])
            assert err < max(1e-12, 10 * e64), (lt, lr, err, e64)
            e_ld = abs(ref["logdet"][0] - ref["logdet_ld"][0])
            assert abs(ld.item() - ref["logdet_ld"][0]) <= max(
                1e-12 * abs(ref["logdet_ld"][0]), 10 * e_ld), (lt, lr)


def test_table_rules(tmp_path):
    # entries apply from their rows bucket up; the largest bucket <= rows wins
    _load(tmp_path, [_line("dnet", ldk.F64, 16, 1, 10, 3), _line("dnet", ldk.F64, 16, 16, 12, 2)])
    assert ldk.plan_info("dnet", ldk.F64, 16, 1)["log_tile"] == 10
    assert ldk.plan_info("dnet", ldk.F64, 16, 15)["log_tile"] == 10
    assert ldk.plan_info("dnet", ldk.F64, 16, 16) == {"log_tile": 12, "radix": 4, "engine": 0,
                                                       "passes": ldk.plan_info("dnet", ldk.F64,
                                                                               16, 16)["passes"]}
    assert ldk.plan_info("dnet", ldk.F64, 17, 16)["log_tile"] == 12  # default elsewhere
    # a bad file leaves the table as it was
    p = tmp_path / "bad.txt"
    for text in ("1 0 16 0 13 3\n", "1 0 16 0 10\n", "5 0 16 0 10 3\n", "0 0 20 0 12 1\n"):
        p.write_text(text)
        with pytest.raises(ldk.LdkError):
            ldk.load_tuned(str(p))
        assert ldk.plan_info("dnet", ldk.F64, 16, 1)["log_tile"] == 10
    with pytest.raises(ldk.LdkError):
        ldk.load_tuned(str(tmp_path / "missing.txt"))
    # workspaces cover every plan the table may choose
    ldk.load_tuned(None)
    base = ldk.lib().ldk_workspace_bytes(ldk.OP_SOLVE, 0, 4, 12, ldk.F64)
    _load(tmp_path, [_line("lattice", ldk.F64, 12, 8, 9, 3)])
    assert ldk.lib().ldk_workspace_bytes(ldk.OP_SOLVE, 0, 4, 12, ldk.F64) >= base
    assert ldk.plan_info("lattice", ldk.F64, 12, 8)["passes"] > 1
    assert ldk.lib().ldk_workspace_bytes(ldk.OP_SOLVE, 0, 4, 12, ldk.F64) > 0


def test_tuner_writes_a_loadable_table(tmp_path):
    from paper_2502_14256_amd import tune
    out = tmp_path / "tuned.txt"
    res = tune.tune([("dnet", ldk.F64, 14, 4, "solve"), ("lattice", ldk.F64, 13, 2, "eig"),
                     ("dnet", ldk.F32, 13, 4, "solve"), ("dnet", ldk.F32, 12, 2, "mll")],
                    K=3, out=str(out), verbose=False)
    assert len(res) == 4 and all(len(r[1]) >= 2 for r in res)
    # the FP32 net cases time the matrix-core engine as one candidate
    assert all(any(t[2] == 1 for t in r[1]) for r in res[2:])
    ldk.load_tuned(str(out))
    for (case, timings, best) in res:
        kind, dt, m, rows, _ = case
        info = ldk.plan_info(kind, dt, m, rows)
        assert info["engine"] == best[2]
        if best[2] == 0:
            assert info["log_tile"] == best[0]


def test_committed_table_loads():
    path = os.path.join(os.path.dirname(ldk.__file__), "tuned_mi355x.txt")
    if not os.path.exists(path):
        pytest.skip("no tuned table committed")
    ldk.load_tuned(path)
