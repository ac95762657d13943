"""ldk_solve_noalloc (the solve whose intermediates live in the library's
fixed per-GPU scratch, for callers that cannot allocate) against ldk_solve
with a caller workspace: bit for bit on two calls in a row, the second with
a smaller input, plus the refusal of inputs beyond the scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2502_14256_amd as ldk

pytestmark = pytest.mark.gpu


def _case(kind, m, R, nrhs, dtype, seed):
    rng = np.random.default_rng(seed)
    n = 2**m
    lam = torch.from_numpy(1.0 + rng.random((R, n))).cuda()
    y = torch.from_numpy(rng.standard_normal((R, nrhs, n))).to(dtype).cuda()
    return lam, y


def _noalloc_call(kind, lam, s2, y, out):
    """Straight through the C ABI."""
    R, nrhs, n = y.shape
    m = n.bit_length() - 1
    dt = ldk.F64 if y.dtype == torch.float64 else ldk.F32
    return ldk.lib().ldk_solve_noalloc(ldk._kind(kind), R, nrhs, m, dt, C.c_void_p(lam.data_ptr()),
                                       float(s2), C.c_void_p(y.data_ptr()),
                                       C.c_void_p(out.data_ptr()),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("kind,dtype", [("lattice", torch.float64), ("lattice", torch.float32),
                                        ("dnet", torch.float64)])
def test_noalloc_solve_matches_solve_twice(kind, dtype):
    ldk.init()
    s2 = 1e-3
    # first call: the largest FP64 lattice of one right-hand side at n = 2^20
    # (8 MiB of intermediates); second call: a smaller input
    for m, R, nrhs, seed in ((20, 1, 1, 1), (15, 2, 3, 2)):
        lam, y = _case(kind, m, R, nrhs, dtype, seed)
        want = ldk.solve(kind, lam, s2, y)
        got = torch.full_like(y, float("nan"))
        rc = _noalloc_call(kind, lam, s2, y, got)
        assert rc == 0, ldk.lib().ldk_strerror(rc)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (m, R, nrhs)


def test_noalloc_solve_refuses_inputs_beyond_the_scratch():
    ldk.init()
    # FP64 lattice, two right-hand sides at n = 2^21: 32 MiB of intermediates
    lam, y = _case("lattice", 21, 1, 2, torch.float64, 3)
    out = torch.full_like(y, 7.0)
    assert _noalloc_call("lattice", lam, 1e-3, y, out) == -5  # LDK_ETOOBIG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing enqueued
    with pytest.raises(ldk.LdkError, match="status -5"):
        ldk.solve_noalloc("lattice", lam, 1e-3, y, out)
    # and the binding's wrapper agrees with ldk_solve on an input that fits
    lam, y = _case("lattice", 12, 3, 2, torch.float64, 4)
    got = ldk.solve_noalloc("lattice", lam, 1e-3, y, torch.empty_like(y))
    assert torch.equal(got, ldk.solve("lattice", lam, 1e-3, y))
