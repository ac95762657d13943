"""Batched fit over an instance table of mixed kind and size: every
instance's solution and log-det equal the one-instance calls bit for bit,
stay within the end-to-end gate of the oracle, and a captured graph of the
whole table replays to the same values."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from paper_2502_14256_amd.batch import BatchFit, Instance
from ldk_dev import kernel, pointset, rel

pytestmark = pytest.mark.gpu

MS = [3, 3, 9, 9, 9, 12, 13, 13, 13, 0, 1]
KINDS = ["lattice", "dnet", "lattice", "dnet", "lattice", "dnet", "lattice", "dnet", "lattice",
         "dnet", "lattice"]


@pytest.fixture(scope="module")
def table():
    return W.small_batch(21, MS, KINDS, d=5, nrhs=3, m_max=13)


def _instances(t, dtype=np.float64):
    return [Instance(kind=ins["kind"], m=ins["m"], shift=ins["shift"][0],
                     lms=None if ins["lms"] is None else ins["lms"][0],
                     y=ins["y"][0].astype(dtype)) for ins in t["instances"]]


def _batch(t, dtype=torch.float64):
    return BatchFit(_instances(t), {"lattice": t["lattice_gen"], "dnet": t["net_gen"]},
                    t["m_max"], t["alpha"], t["gamma"], t["zeta"], t["sigma2"], dtype=dtype)


def _single(t, i, dtype=torch.float64):
    w = W.instance_workload(t, i)
    ps, k = pointset(w), kernel(w)
    n = 2 ** w["m"]
    k1 = ldk.kernel_column(k, ps, 0, n, dtype=dtype)
    lam = ldk.eig(w["kind"], k1)
    c = ldk.solve(w["kind"], lam, w["sigma2"], torch.from_numpy(w["y"]).cuda().to(dtype))
    ld = ldk.logdet(lam, w["sigma2"])
    return c[0], ld[0]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_equals_single_calls(table, dtype):
    b = _batch(table, dtype)
    assert len(b.groups) == len(set(zip(MS, KINDS)))
    b.step()
    for i in range(len(MS)):
        c, ld = b.result(i)
        c1, ld1 = _single(table, i, dtype)
        assert torch.equal(c, c1), i
        assert torch.allclose(ld, ld1, rtol=1e-13, atol=1e-12, equal_nan=True), i


def test_plain_step_equals_batched(table):
    b = _batch(table)
    b.step()
    ref = [tuple(t.clone() for t in b.result(i)) for i in range(len(MS))]
    b.step_plain()
    for i in range(len(MS)):
        c, ld = b.result(i)
        # the batched step fits with ldk_fit: the same solutions, the log-det
        # summed in another fixed order
        assert torch.equal(c, ref[i][0]), i
        assert torch.allclose(ld, ref[i][1], rtol=1e-13, atol=1e-12), i


def test_batched_matches_oracle(table):
    import oracle
    b = _batch(table)
    b.step()
    for i in range(len(MS)):
        w = W.instance_workload(table, i)
        ref = oracle.fit_solve(w, y=w["y"], precise=True)
        c, ld = b.result(i)
        e64 = rel(ref["c"], ref["c_ld"])
        err = rel(c.cpu().numpy()[None], ref["c_ld"])
        assert err < max(1e-12, 10 * e64), (i, err, e64)
        e64_ld = abs(ref["logdet"][0] - ref["logdet_ld"][0])
        assert abs(ld.item() - ref["logdet_ld"][0]) <= max(1e-12 * abs(ref["logdet_ld"][0]),
                                                           10 * e64_ld), i


def test_batched_graph_replays(table):
    b = _batch(table)
    g = b.capture()
    torch.cuda.synchronize()
    ref = [tuple(t.clone() for t in b.result(i)) for i in range(len(MS))]
    for rep in range(3):
        for grp in b.groups:
            grp["c"].fill_(-1)
            grp["ld"].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(MS)):
            c, ld = b.result(i)
            assert torch.equal(c, ref[i][0]) and torch.equal(ld, ref[i][1]), (rep, i)
