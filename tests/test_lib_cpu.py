"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/ldk.h declares, and rejects invalid arguments
before enqueueing anything."""
import ctypes as C
import os
import re

import pytest

import paper_2502_14256_amd as ldk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ldk.h")).read()
    return sorted(set(re.findall(r"\b(ldk_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(ldk.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ldk.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_strerror():
    L = ldk.lib()
    assert L.ldk_version().decode().count(".") == 2
    for code in (0, -1, -2, -3, -4):
        assert L.ldk_strerror(code).decode()
    assert L.ldk_strerror(-99).decode() == "unknown status"


FAKE = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def _ps(**kw):
    base = dict(kind=ldk.DNET_B2, order=ldk.NATURAL, R=1, d=4, m_max=10, flags=0,
                gen=FAKE, lms=None, shift=None)
    base.update(kw)
    return ldk._Pointset(**base)


@pytest.mark.parametrize("kw", [
    dict(R=0), dict(d=0), dict(d=5000), dict(m_max=63), dict(kind=7), dict(gen=None),
    dict(order=ldk.LINEAR), dict(kind=ldk.LATTICE, order=ldk.GRAY),
    dict(kind=ldk.LATTICE, lms=FAKE),
])
def test_gen_points_rejects_bad_pointsets(kw):
    L = ldk.lib()
    assert L.ldk_gen_points(C.byref(_ps(**kw)), 0, 4, FAKE, None) == -1


def test_gen_points_rejects_bad_ranges():
    L = ldk.lib()
    assert L.ldk_gen_points(C.byref(_ps()), 5, 4, FAKE, None) == -1
    assert L.ldk_gen_points(C.byref(_ps()), -1, 4, FAKE, None) == -1
    assert L.ldk_gen_points(C.byref(_ps()), 0, 2**10 + 1, FAKE, None) == -1  # beyond 2^m_max
    assert L.ldk_gen_points(C.byref(_ps()), 0, 4, None, None) == -1
    # empty range: valid, nothing to do
    assert L.ldk_gen_points(C.byref(_ps()), 3, 3, FAKE, None) == 0


def _alpha(*vals):
    arr = (C.c_int32 * len(vals))(*vals)
    return arr, C.cast(arr, C.c_void_p)


def test_kernel_column_rejects_mismatch():
    L = ldk.lib()
    keep, a4 = _alpha(2, 2, 2, 2)
    k = ldk._Kernel(ldk.LATTICE, 4, a4, FAKE, 1.0)
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, FAKE, None) == -1
    k = ldk._Kernel(ldk.DNET_B2, 4, a4, FAKE, 0.0)  # zeta must be > 0
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, FAKE, None) == -1
    k = ldk._Kernel(ldk.DNET_B2, 4, a4, FAKE, 1.0)
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), None, None, 0, 4, 9, FAKE, None) == -1
    # pts given with n_min > 0 needs an explicit anchor
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), FAKE, None, 2, 4, 0, FAKE, None) == -1
    # orders are validated on the host: nets 1..4, lattices 1..3
    keep5, bad = _alpha(1, 2, 5, 1)
    k = ldk._Kernel(ldk.DNET_B2, 4, bad, FAKE, 1.0)
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, FAKE, None) == -1
    keep4, bad4 = _alpha(1, 4, 2, 1)
    k = ldk._Kernel(ldk.LATTICE, 4, bad4, FAKE, 1.0)
    ps = _ps(kind=ldk.LATTICE)
    assert L.ldk_kernel_column(C.byref(k), C.byref(ps), None, None, 0, 4, 0, FAKE, None) == -1
    keep0, bad0 = _alpha(1, 0, 2, 1)
    k = ldk._Kernel(ldk.DNET_B2, 4, bad0, FAKE, 1.0)
    assert L.ldk_kernel_column(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, FAKE, None) == -1


def test_points_column_rejects_bad_arguments():
    L = ldk.lib()
    keep, a4 = _alpha(2, 2, 2, 2)
    k = ldk._Kernel(ldk.DNET_B2, 4, a4, FAKE, 1.0)
    ps = _ps()
    f = L.ldk_points_column
    assert f(None, C.byref(ps), 0, 4, FAKE, 0, FAKE, None) == -1
    assert f(C.byref(k), None, 0, 4, FAKE, 0, FAKE, None) == -1
    assert f(C.byref(k), C.byref(ps), 0, 4, FAKE, 9, FAKE, None) == -1      # dtype
    assert f(C.byref(k), C.byref(ps), 5, 4, FAKE, 0, FAKE, None) == -1      # n_max < n_min
    assert f(C.byref(k), C.byref(ps), -1, 4, FAKE, 0, FAKE, None) == -1
    assert f(C.byref(k), C.byref(ps), 0, 2**10 + 1, FAKE, 0, FAKE, None) == -1  # beyond 2^m_max
    assert f(C.byref(k), C.byref(ps), 0, 4, None, 0, FAKE, None) == -1      # no points buffer
    assert f(C.byref(k), C.byref(ps), 0, 4, FAKE, 0, None, None) == -1      # no column buffer
    kl = ldk._Kernel(ldk.LATTICE, 4, a4, FAKE, 1.0)
    assert f(C.byref(kl), C.byref(ps), 0, 4, FAKE, 0, FAKE, None) == -1     # kind mismatch
    # empty window: valid, nothing to do, the outputs may be NULL
    assert f(C.byref(k), C.byref(ps), 3, 3, None, 0, None, None) == 0


def test_interlace_and_flags_reject_bad_arguments():
    L = ldk.lib()
    # flags: only LDK_GEN_PER_REPLICATION, and only for nets
    assert L.ldk_gen_points(C.byref(_ps(flags=2)), 0, 4, FAKE, None) == -1
    assert L.ldk_gen_points(C.byref(_ps(kind=ldk.LATTICE, flags=1)), 0, 4, FAKE, None) == -1
    f = L.ldk_interlace
    assert f(C.byref(_ps(d=4)), 0, FAKE, None) == -1        # alpha < 1
    assert f(C.byref(_ps(d=4)), 5, FAKE, None) == -1        # alpha > 4
    assert f(C.byref(_ps(d=6)), 4, FAKE, None) == -1        # d not a multiple of alpha
    assert f(C.byref(_ps(kind=ldk.LATTICE)), 2, FAKE, None) == -1
    assert f(C.byref(_ps(flags=1)), 2, FAKE, None) == -1    # source columns must be shared
    assert f(C.byref(_ps(d=4)), 2, None, None) == -1        # no output
    assert f(None, 2, FAKE, None) == -1
    # a net without columns (m_max = 0): nothing to write
    assert f(C.byref(_ps(d=4, m_max=0, gen=None)), 2, None, None) == 0


def test_algebra_rejects_bad_arguments():
    L = ldk.lib()
    assert L.ldk_transform(5, 1, 1, 4, 0, FAKE, FAKE, None, None) == -1
    assert L.ldk_transform(ldk.LATTICE, 0, 1, 4, 0, FAKE, FAKE, None, None) == -1
    assert L.ldk_transform(ldk.DNET_B2, 1, 1, 27, 0, FAKE, FAKE, None, None) == -1
    assert L.ldk_transform(ldk.DNET_B2, 1, 1, 4, 3, FAKE, FAKE, None, None) == -1
    assert L.ldk_transform(ldk.DNET_B2, 1, 0, 4, 0, FAKE, FAKE, None, None) == 0  # B = 0
    assert L.ldk_solve(ldk.DNET_B2, 1, 1, 4, 0, FAKE, -1.0, FAKE, FAKE, None, None) == -1
    assert L.ldk_solve(ldk.DNET_B2, 1, 1, 4, 0, None, 0.1, FAKE, FAKE, None, None) == -1
    assert L.ldk_solve(ldk.DNET_B2, 0, 1, 4, 0, FAKE, 0.1, FAKE, FAKE, None, None) == 0
    # lattice solve with more than one pass needs its workspace
    assert L.ldk_solve(ldk.LATTICE, 1, 1, 20, 0, FAKE, 0.1, FAKE, FAKE, None, None) == -1
    assert L.ldk_logdet(1, 4, FAKE, 0.1, FAKE, None, None) == -1  # workspace missing
    assert L.ldk_logdet(1, 4, FAKE, float("nan"), FAKE, FAKE, None) == -1
    assert L.ldk_update_double(ldk.DNET_B2, 1, 26, 0, FAKE, FAKE, FAKE, None, None) == -1
    assert L.ldk_eig(ldk.LATTICE, 1, 20, 0, FAKE, FAKE, None, None) == -1


def test_workspace_sizes():
    L = ldk.lib()
    ws = L.ldk_workspace_bytes
    assert ws(ldk.OP_TRANSFORM, ldk.DNET_B2, 4, 20, 0) == 0
    assert ws(ldk.OP_SOLVE, ldk.DNET_B2, 4, 20, 0) == 0
    # real lattice rows of n run as packed complex rows of n/2, plus the
    # solve filter's coefficients for up to B / 2 eigenvalue rows
    assert ws(ldk.OP_SOLVE, ldk.LATTICE, 4, 20, 0) == (4 + 2) * 2**19 * 16
    assert ws(ldk.OP_SOLVE, ldk.LATTICE, 4, 20, 1) == (4 + 2) * 2**19 * 8
    assert ws(ldk.OP_SOLVE, ldk.LATTICE, 1, 20, 0) == 2**19 * 16
    assert ws(ldk.OP_SOLVE, ldk.LATTICE, 4, 10, 0) == 0  # one pass, no intermediate
    assert ws(ldk.OP_LOGDET, ldk.DNET_B2, 3, 20, 0) == 3 * 512 * 8
    assert ws(ldk.OP_EIG, 9, 1, 4, 0) == 0
    # eigenvalue transforms run in FP64 whatever the input dtype
    assert ws(ldk.OP_EIG, ldk.LATTICE, 2, 20, 1) == 2 * 2**19 * 16
    assert ws(ldk.OP_EIG, ldk.LATTICE, 2, 12, 0) == 0  # n/2 = 2^11 fits one pass


def test_likelihood_entry_points_reject_bad_arguments():
    L = ldk.lib()
    # ldk_mll(kind, R, m, dtype, lam, sigma2, y, L, g, dlogs2, ws, stream)
    assert L.ldk_mll(7, 1, 4, 0, FAKE, 0.1, FAKE, FAKE, FAKE, None, FAKE, None) == -1
    assert L.ldk_mll(ldk.LATTICE, 1, 4, 5, FAKE, 0.1, FAKE, FAKE, FAKE, None, FAKE, None) == -1
    assert L.ldk_mll(ldk.LATTICE, 1, 27, 0, FAKE, 0.1, FAKE, FAKE, FAKE, None, FAKE, None) == -1
    assert L.ldk_mll(ldk.DNET_B2, 1, 4, 0, FAKE, -1.0, FAKE, FAKE, FAKE, None, FAKE, None) == -1
    assert L.ldk_mll(ldk.DNET_B2, 1, 4, 0, FAKE, float("nan"), FAKE, FAKE, FAKE, None, FAKE,
                     None) == -1
    assert L.ldk_mll(ldk.DNET_B2, 1, 4, 0, FAKE, 0.1, FAKE, FAKE, FAKE, None, None, None) == -1
    assert L.ldk_mll(ldk.DNET_B2, 1, 4, 0, None, 0.1, FAKE, FAKE, FAKE, None, FAKE, None) == -1
    assert L.ldk_mll(ldk.DNET_B2, 0, 4, 0, None, 0.1, None, None, None, None, None, None) == 0
    # ldk_mll_adjoint(kind, R, m, g, a, ws, stream)
    assert L.ldk_mll_adjoint(7, 1, 4, FAKE, FAKE, None, None) == -1
    assert L.ldk_mll_adjoint(ldk.LATTICE, 1, 4, None, FAKE, None, None) == -1
    assert L.ldk_mll_adjoint(ldk.LATTICE, 1, 20, FAKE, FAKE, None, None) == -1  # needs ws
    assert L.ldk_mll_adjoint(ldk.LATTICE, 0, 20, None, None, None, None) == 0
    # ldk_kernel_grad: the kernel-column validation, then a, grad and ws
    keep, a4 = _alpha(2, 2, 2, 2)
    k = ldk._Kernel(ldk.LATTICE, 4, a4, FAKE, 1.0)  # kind mismatch with the net point set
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, None, FAKE, FAKE, FAKE,
                             None) == -1
    k = ldk._Kernel(ldk.DNET_B2, 4, a4, FAKE, 1.0)
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, None, FAKE, None, FAKE,
                             None) == -1  # grad missing
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, None, None, FAKE, FAKE,
                             None) == -1  # a missing
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, None, FAKE, FAKE, None,
                             None) == -1  # ws missing
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 2**10 + 1, 0, None, FAKE,
                             FAKE, FAKE, None) == -1  # beyond 2^m_max
    keep5, bad = _alpha(1, 2, 5, 1)
    k = ldk._Kernel(ldk.DNET_B2, 4, bad, FAKE, 1.0)
    assert L.ldk_kernel_grad(C.byref(k), C.byref(_ps()), None, None, 0, 4, 0, None, FAKE, FAKE, FAKE,
                             None) == -1


def test_likelihood_workspace_sizes():
    L = ldk.lib()
    ws = L.ldk_workspace_bytes
    # partial sums (3 doubles per 2048 entries, 256-byte aligned) + transform scratch
    assert ws(ldk.OP_MLL, ldk.DNET_B2, 2, 10, 0) == 256  # one pass: partials only
    assert ws(ldk.OP_MLL, ldk.DNET_B2, 2, 20, 0) == 2 * 512 * 3 * 8 + 2 * 2**20 * 8
    assert ws(ldk.OP_MLL, ldk.LATTICE, 2, 20, 1) == 2 * 512 * 3 * 8 + 2 * 2**19 * 8
    assert ws(ldk.OP_MLL_ADJOINT, ldk.DNET_B2, 2, 20, 0) == 0
    assert ws(ldk.OP_MLL_ADJOINT, ldk.LATTICE, 2, 20, 0) == 2 * 2**19 * 16
    assert ws(ldk.OP_MLL_ADJOINT, ldk.LATTICE, 2, 12, 0) == 0
    g = L.ldk_kernel_grad_workspace_bytes
    # [R][tiles of 2048][d + 1] doubles
    assert g(3, 7, 0, 4096, 0) == 3 * 2 * 8 * 8
    assert g(3, 7, 100, 4096, 0) == 3 * 2 * 8 * 8      # tiles aligned to 2048
    assert g(3, 7, 100, 4097, 1) == 3 * 2 * 8 * 8      # tiles from n_min
    assert g(3, 7, 100, 4197, 1) == 3 * 3 * 8 * 8
    assert g(0, 7, 0, 4096, 0) == 0
    assert ws(ldk.OP_MLL, ldk.LATTICE, 3, 0, 0) == 256  # n = 1 still sums


def test_fwht_split16_rejects_bad_arguments():
    L = ldk.lib()
    assert L.ldk_fwht_split16(-1, 4, FAKE, FAKE, None) == -1
    assert L.ldk_fwht_split16(1, 27, FAKE, FAKE, None) == -1
    assert L.ldk_fwht_split16(1, 4, None, FAKE, None) == -1
    assert L.ldk_fwht_split16(0, 4, None, None, None) == 0


def test_cubature_entry_points_reject_bad_arguments():
    L = ldk.lib()
    nan = float("nan")
    # ldk_wce(kind, R, nw, m, dtype, lam, zeta, w, e2, ws, stream)
    f = L.ldk_wce
    assert f(7, 1, 1, 4, 0, FAKE, 1.0, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.LATTICE, 1, 1, 4, 5, FAKE, 1.0, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.LATTICE, 1, 1, 27, 0, FAKE, 1.0, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.DNET_B2, 1, 1, 4, 0, FAKE, nan, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.DNET_B2, 256, 256, 4, 0, FAKE, 1.0, FAKE, FAKE, FAKE, None) == -1  # rows
    assert f(ldk.DNET_B2, 1, -1, 4, 0, FAKE, 1.0, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.DNET_B2, 1, 1, 4, 0, None, 1.0, FAKE, FAKE, FAKE, None) == -1
    assert f(ldk.DNET_B2, 1, 1, 4, 0, FAKE, 1.0, FAKE, FAKE, None, None) == -1   # ws
    assert f(ldk.DNET_B2, 1, 1, 4, 0, FAKE, 1.0, FAKE, None, FAKE, None) == -1   # e2
    assert f(ldk.DNET_B2, 3, 0, 4, 0, None, 1.0, None, None, None, None) == 0    # nothing to do
    assert f(ldk.DNET_B2, 0, 3, 4, 0, None, 1.0, None, None, None, None) == 0
    # ldk_bayes_cubature(kind, R, m, dtype, lam, sigma2, zeta, y, z, out, ws, stream)
    g = L.ldk_bayes_cubature
    assert g(7, 1, 4, 0, FAKE, 0.1, 1.0, FAKE, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, -1.0, 1.0, FAKE, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, nan, 1.0, FAKE, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, 0.1, nan, FAKE, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, 0.1, 1.0, FAKE, -2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 65536, 4, 0, FAKE, 0.1, 1.0, FAKE, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, 0.1, 1.0, None, 2.0, FAKE, FAKE, None) == -1
    assert g(ldk.LATTICE, 1, 4, 0, FAKE, 0.1, 1.0, FAKE, 2.0, FAKE, None, None) == -1
    assert g(ldk.LATTICE, 0, 4, 0, None, 0.1, 1.0, None, 2.0, None, None, None) == 0


def test_cubature_workspace_sizes():
    ws = ldk.lib().ldk_workspace_bytes
    # partial sums (2 doubles per 2048 entries, 256-byte aligned) + power
    # spectrum (FP64 rows) + transform scratch
    assert ws(ldk.OP_WCE, ldk.DNET_B2, 2, 10, 0) == 256 + 2 * 2**10 * 8
    assert ws(ldk.OP_WCE, ldk.DNET_B2, 2, 20, 0) == 2 * 512 * 2 * 8 + 2 * 2**20 * 8 * 2
    assert ws(ldk.OP_BAYES_CUBATURE, ldk.LATTICE, 2, 20, 1) == (2 * 512 * 2 * 8 + 2 * 2**20 * 8
                                                              + 2 * 2**19 * 8)
    assert ws(ldk.OP_BAYES_CUBATURE, ldk.LATTICE, 3, 0, 0) == 256 + 256


def test_rqmc_rejects_bad_arguments():
    L = ldk.lib()
    f = L.ldk_rqmc
    P, CP, OSC = C.byref, ldk.GENZ_CORNER_PEAK, ldk.GENZ_OSCILLATORY
    # ldk_rqmc(ps, n, integrand, coef, u, t, mu_r, stats, ws, stream)
    assert f(P(_ps(R=0)), 16, CP, FAKE, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1
    assert f(P(_ps()), 16, 2, FAKE, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1       # integrand
    assert f(P(_ps()), 0, CP, FAKE, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1       # n >= 1
    assert f(P(_ps()), 2**10 + 1, CP, FAKE, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1  # > 2^m
    assert f(P(_ps()), 16, OSC, FAKE, float("nan"), 2.0, FAKE, FAKE, FAKE, None) == -1
    assert f(P(_ps()), 16, CP, FAKE, 0.0, -1.0, FAKE, FAKE, FAKE, None) == -1     # t >= 0
    assert f(P(_ps()), 16, CP, None, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1      # coef
    assert f(P(_ps()), 16, CP, FAKE, 0.0, 2.0, None, FAKE, FAKE, None) == -1      # mu_r
    assert f(P(_ps()), 16, CP, FAKE, 0.0, 2.0, FAKE, None, FAKE, None) == -1      # stats
    assert f(P(_ps()), 16, CP, FAKE, 0.0, 2.0, FAKE, FAKE, None, None) == -1      # ws
    assert f(None, 16, CP, FAKE, 0.0, 2.0, FAKE, FAKE, FAKE, None) == -1
    # tile sums: R x ceil(n / 512) doubles (room for the small-grid tiling),
    # 256-byte aligned, then the scrambled columns R x d x m_max of an LMS net
    w = L.ldk_rqmc_workspace_bytes
    assert w(P(_ps(kind=ldk.LATTICE, R=10, gen=FAKE)), 2**15) == 10 * 64 * 8
    assert w(P(_ps(kind=ldk.LATTICE, R=3)), 2049) == 256
    assert w(P(_ps(R=3, lms=FAKE)), 2049) == 256 + 3 * 4 * 10 * 8
    assert w(P(_ps(R=3)), 0) == 0
    assert w(P(_ps(R=0)), 16) == 0  # invalid point set
