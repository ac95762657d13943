"""GPU parity of the RQMC estimate and its Student-t interval (eq. RQMC)
against the oracle, for the Genz corner peak and oscillatory integrands on
every kind of point set (shifted lattices in both orders, LMS + digitally
shifted nets in both orders, interlaced higher-order nets), at ragged sizes,
at the paper's example shape (d = 50, n = 2^15, R = 10, order-3 interlaced
net) and at n = 2^20."""
import math

import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import U64_EPS, dev_u64, pointset, record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _ref(orc, pts, integrand, c, u, tau):
    x = orc.unit_points(pts)
    y = orc.genz_corner_peak(x, c) if integrand == "corner_peak" else \
        orc.genz_oscillatory(x, c, u)
    return orc.rqmc(y, tau=tau), y


def _check(name, mu_r, stats, ref, y, integrand, c, n):
    """Derived bounds: s = c.x summed in another order (|ds| <= 2 d u sum|c x|);
    the corner peak's relative error (d + 1)|ds|/(1 + s) plus its power
    (binary powering here, (d + 2) u; pow in the oracle), the oscillatory's
    absolute error |ds| plus its cosine; then the FP64 sums of n terms (tree
    depth log2 n on both sides)."""
    u = U64_EPS
    d = len(c)
    R = mu_r.shape[0]
    absf = np.abs(y).mean(axis=1)
    if integrand == "corner_peak":
        f_err = (2 * d * (d + 1) + (d + 2) + 8) * u * absf
    else:
        f_err = (2 * d * np.abs(c).sum() + 4) * u
    tol_mu = 4 * (f_err + (2 * math.log2(max(n, 2)) + 20) * u * absf)
    e_mu = np.abs(mu_r - ref["mu_r"]) / tol_mu
    tol_mean = tol_mu.max() + 4 * R * u * np.abs(ref["mu_r"]).max()
    e_mean = abs(stats[0] - ref["mean"]) / tol_mean
    errs = dict(mu_r=e_mu.max(), mean=e_mean)
    if R > 1:
        tol_std = 2 * math.sqrt(R / (R - 1)) * tol_mean + 8 * R * u * ref["std"]
        errs["std"] = abs(stats[1] - ref["std"]) / tol_std
        tol_half = ref["t"] * tol_std / math.sqrt(R) + 8 * u * ref["half"]
        errs["half"] = abs(stats[2] - ref["half"]) / tol_half
    else:
        assert np.isnan(stats[1]) and np.isnan(stats[2])
    record(name, **{f"{k}_over_tol": v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= 1.0, (k, v, mu_r, ref)


def _run(ps, n, integrand, c, u=0.37, tau=0.01):
    coef = torch.from_numpy(np.asarray(c, np.float64)).cuda()
    mu_r, stats = ldk.rqmc(ps, n, integrand, coef, u=u, tau=tau)
    return mu_r.cpu().numpy(), stats.cpu().numpy()


CASES = [  # kind, order, lms, d, m, R, n
    ("lattice", "natural", False, 3, 12, 2, 2**12),
    ("lattice", "natural", False, 5, 14, 3, 5000),
    ("lattice", "natural", False, 1, 4, 1, 1),
    ("lattice", "linear", False, 4, 13, 2, 2**13),
    ("lattice", "linear", False, 2, 13, 2, 2049),
    ("dnet", "natural", True, 3, 12, 2, 2**12),
    ("dnet", "natural", True, 9, 13, 3, 3001),
    ("dnet", "gray", True, 5, 12, 2, 2**12),
    ("dnet", "gray", False, 17, 11, 2, 777),
    ("dnet", "natural", False, 2, 0, 2, 1),
]


@pytest.mark.parametrize("integrand", ["corner_peak", "oscillatory"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_rqmc_parity(orc, integrand, case):
    kind, order, lms, d, m, R, n = case
    w = W.small_lattice(200 + d, m, d, R) if kind == "lattice" else W.small_net(200 + d, m, d, R)
    if not lms:
        w["lms"] = None
    w["order"] = order
    c = np.random.default_rng(d).uniform(0.1, 1.2, d) if integrand == "oscillatory" \
        else W.corner_peak_coefficients(d)
    pts = orc.points(w, 0, n, order)
    ref, y = _ref(orc, pts, integrand, c, 0.37, 0.01)
    mu_r, stats = _run(pointset(w, order), n, integrand, c)
    _check(f"rqmc_{integrand}_{'-'.join(map(str, case))}", mu_r, stats, ref, y, integrand, c, n)


# Enough tiles of 8 points per thread (n R >= 2^20) that the kernel takes
# that form, with ragged ends of the last tile
CASES_IT8 = [  # kind, order, lms, d, m, R, n
    ("lattice", "natural", False, 7, 18, 5, 2**18 - 1000),
    ("lattice", "linear", False, 3, 18, 4, 2**18),
    ("dnet", "natural", True, 7, 18, 5, 2**18 - 1000),
    ("dnet", "gray", True, 5, 18, 4, 2**18),
]


@pytest.mark.parametrize("case", CASES_IT8, ids=lambda c: "-".join(map(str, c)))
def test_rqmc_parity_eight_per_thread(orc, case):
    test_rqmc_parity(orc, "corner_peak", case)


def _paper_shape(R=10, d=50, m=15, alpha=3, order="natural"):
    src = W.small_net(2502, m=m, d=alpha * d, R=R)
    shift = np.random.default_rng(7).integers(0, 2**64, size=(R, d), dtype=np.uint64)
    ps_src = ldk.PointSet("dnet", R, alpha * d, m, dev_u64(src["gen"]), dev_u64(src["lms"]), None,
                          order=order)
    return src, shift, ps_src


@pytest.mark.parametrize("order", ["natural", "gray"])
def test_rqmc_paper_example_shape(orc, order):
    # corner peak, d = 50, n = 2^15, R = 10, order-3 interlaced LMS + shifted net
    d, m, R, alpha = 50, 15, 10, 3
    src, shift, ps_src = _paper_shape(R, d, m, alpha, order)
    hp = ldk.interlace(ps_src, alpha, shift=dev_u64(shift))
    c = W.corner_peak_coefficients(d)
    pts = orc.higher_order_dnet_points(src["gen"], src["lms"], shift, alpha, m, 0, 2**m, order)
    ref, y = _ref(orc, pts, "corner_peak", c, 0.0, 0.01)
    mu_r, stats = _run(hp, 2**m, "corner_peak", c)
    _check(f"rqmc_paper_shape_{order}", mu_r, stats, ref, y, "corner_peak", c, 2**m)
    # the estimate sits near the paper's printed one (0.0149368) at the
    # precision of its own interval
    assert abs(stats[0] - 0.014936813948394042) <= max(2 * stats[2], 2e-6)


def test_rqmc_full_size(orc):
    # n = 2^20 shifted lattice in natural order, d = 50, one replication
    d, m, R = 50, 20, 1
    w = W.small_lattice(2505, m, d, R)
    c = W.corner_peak_coefficients(d)
    pts = orc.points(w)
    ref, y = _ref(orc, pts, "corner_peak", c, 0.0, 0.01)
    del pts
    mu_r, stats = _run(pointset(w), 2**m, "corner_peak", c)
    _check("rqmc_full_lattice_m20_d50", mu_r, stats, ref, y, "corner_peak", c, 2**m)


def test_rqmc_identical_replications(orc):
    # R copies of one randomization: every mu_r is bit-identical, std and half are 0
    d, m, R = 6, 12, 4
    w = W.small_net(300, m, d, 1)
    w["lms"] = np.repeat(w["lms"], R, axis=0)
    w["shift"] = np.repeat(w["shift"], R, axis=0)
    w["R"] = R
    mu_r, stats = _run(pointset(w), 2**m, "corner_peak", W.corner_peak_coefficients(d))
    assert np.all(mu_r == mu_r[0])
    assert stats[1] == 0.0 and stats[2] == 0.0


@pytest.mark.parametrize("order", ["natural", "gray"])
def test_rqmc_per_replication_columns_with_lms(orc, order):
    # a net whose generating columns differ per replication (flags =
    # LDK_GEN_PER_REPLICATION) and that also carries LMS scrambles: each
    # replication's points are the LMS net of its own columns
    d, m, R, n = 6, 12, 3, 3000
    rng = np.random.default_rng(88)
    cols = np.stack([W.net_generating_matrices(rng, d, m) for _ in range(R)])
    S = W.lms_matrices(rng, R, d)
    shift = W.shifts(rng, R, d)
    ps = ldk.PointSet("dnet", R, d, m, dev_u64(cols), dev_u64(S), dev_u64(shift), order=order,
                      per_replication=True)
    pts = np.stack([orc.dnet_points(cols[r], S[r:r + 1], shift[r:r + 1], m, 0, n, order, R=1)[0]
                    for r in range(R)])
    c = W.corner_peak_coefficients(d)
    ref, y = _ref(orc, pts, "corner_peak", c, 0.0, 0.01)
    mu_r, stats = _run(ps, n, "corner_peak", c, u=0.0)
    _check(f"rqmc_per_rep_lms_{order}", mu_r, stats, ref, y, "corner_peak", c, n)
