"""HIP-graph capture of a whole fit + solve step: several replays, with eager
work and synchronisations between them, each checked bit for bit against the
eager result (the library records no memset and no allocation)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import kernel, pointset

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("branches", [False, True])
def test_graph_replays_match_eager(kind, branches):
    ldk.init()
    m, d, R = 16, 8, 2
    w = W.small_lattice(3, m=m, d=d, R=R) if kind == "lattice" else W.small_net(3, m=m, d=d, R=R)
    w.update(alpha=np.full(d, 2, np.int32), gamma=0.5 ** np.arange(d), zeta=1.0)
    ps, k = pointset(w), kernel(w)
    n = 2**m
    y = torch.from_numpy(w["y"]).cuda()
    pts = torch.empty((R, n, d), dtype=torch.int64, device="cuda")
    k1 = torch.empty((R, n), dtype=torch.float64, device="cuda")
    lam = torch.empty((R, n), dtype=torch.float64, device="cuda")
    c = torch.empty_like(y)
    ld = torch.empty(R, dtype=torch.float64, device="cuda")
    kd = ldk._kind(kind)
    ws_e = ldk._workspace(ldk.OP_EIG, kd, R, m, ldk.F64, "cuda")
    ws_s = ldk._workspace(ldk.OP_SOLVE, kd, R, m, ldk.F64, "cuda")
    ws_l = ldk._workspace(ldk.OP_LOGDET, kd, R, m, ldk.F64, "cuda")

    s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
    ev = torch.cuda.Event()

    def step():
        if not branches:
            ldk.gen_points(ps, 0, n, out=pts)
            ldk.kernel_column(k, ps, 0, n, out=k1)
            ldk.eig(kind, k1, out=lam, ws=ws_e)
            ldk.solve(kind, lam, 1e-4, y, out=c, ws=ws_s)
            ldk.logdet(lam, 1e-4, out=ld, ws=ws_l)
            return
        # points on a side branch; log-det beside the solve (as the benchmark)
        main = torch.cuda.current_stream()
        s_a.wait_stream(main)
        s_b.wait_stream(main)
        with torch.cuda.stream(s_a):
            ldk.gen_points(ps, 0, n, out=pts)
        ldk.kernel_column(k, ps, 0, n, out=k1)
        ldk.eig(kind, k1, out=lam, ws=ws_e)
        ev.record(main)
        with torch.cuda.stream(s_b):
            s_b.wait_event(ev)
            ldk.logdet(lam, 1e-4, out=ld, ws=ws_l)
        ldk.solve(kind, lam, 1e-4, y, out=c, ws=ws_s)
        main.wait_stream(s_a)
        main.wait_stream(s_b)

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (pts, k1, lam, c, ld)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        for t in (pts, k1, lam, c, ld):
            t.fill_(-1)  # eager work between replays; outputs must be rewritten
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((pts, k1, lam, c, ld), ref):
            assert torch.equal(a, b), rep


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_graph_replays_cubature_and_rqmc(kind):
    # the cubature and RQMC entry points captured in one graph: every replay,
    # with eager writes between replays, equals the eager result bit for bit
    ldk.init()
    m, d, R, nw = 14, 6, 3, 4
    w = W.small_lattice(5, m=m, d=d, R=R) if kind == "lattice" else W.small_net(5, m=m, d=d, R=R)
    w.update(alpha=np.full(d, 2, np.int32), gamma=0.5 ** np.arange(d), zeta=1.2)
    ps, k = pointset(w), kernel(w)
    n = 2**m
    y = torch.from_numpy(w["y"][:, 0, :]).cuda()
    k1 = ldk.kernel_column(k, ps, 0, n)
    lam = ldk.eig(kind, k1)
    om = torch.from_numpy(W.cubature_weights(6, R, nw, n)).cuda()
    coef = torch.from_numpy(W.corner_peak_coefficients(d)).cuda()
    kd = ldk._kind(kind)
    e2 = torch.empty((R, nw), dtype=torch.float64, device="cuda")
    bc = torch.empty((R, len(ldk.BC_FIELDS)), dtype=torch.float64, device="cuda")
    mu_r = torch.empty(R, dtype=torch.float64, device="cuda")
    st = torch.empty(3, dtype=torch.float64, device="cuda")
    ws_w = ldk._workspace(ldk.OP_WCE, kd, R * nw, m, ldk.F64, "cuda")
    ws_b = ldk._workspace(ldk.OP_BAYES_CUBATURE, kd, R, m, ldk.F64, "cuda")
    ws_q = torch.empty(int(ldk.lib().ldk_rqmc_workspace_bytes(ctypes.byref(ps._c()), n)),
                       dtype=torch.uint8,
                       device="cuda")

    def step():
        ldk.wce(kind, lam, om, 1.2, out=e2, ws=ws_w)
        ldk.bayes_cubature(kind, lam, 1e-3, 1.2, y, out=bc, ws=ws_b)
        ldk.rqmc(ps, n, "corner_peak", coef, mu_r=mu_r, stats=st, ws=ws_q)

    step()
    torch.cuda.synchronize()
    outs = (e2, bc, mu_r, st)
    ref = [t.clone() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        for t in outs:
            t.fill_(-1)
        ws_w.fill_(7)  # stale workspace contents must not leak into results
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
