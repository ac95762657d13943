"""GPU parity of the point sets without fast-transform structure (Secs. 4.3,
4.4): Halton and Faure coordinates with every combination of LMS, digit
permutations and digital shift, and nested uniform scrambling of a base-2
net, bit for bit against the oracle (both sides form the integer digit value
exactly and divide once, or convert the 64-bit word once); ragged windows,
the largest Halton dimension and the paper's Faure shape (d = 52, b = 53);
argument checks; and the RQMC estimate over these points
(ldk_rqmc_points) against the oracle with the RQMC gates."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_2502_14256_amd as ldk
from ldk_dev import dev_u64

pytestmark = pytest.mark.gpu

FLAG_SETS = [0, 1, 2, 4, 1 | 2, 1 | 4, 1 | 2 | 4]


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _bps(kind, R, d, base=0, flags=0, seed=3):
    inp = W.bpoint_inputs(seed, kind, R, d, base=base)
    dev = {k: torch.from_numpy(v).cuda() for k, v in inp.items()}
    return inp, ldk.BPointSet(kind, R, d, base=base, flags=flags, **dev)


@pytest.mark.parametrize("flags", FLAG_SETS)
@pytest.mark.parametrize("window", [(0, 1000), (37, 1234)])
def test_halton_bit_exact(orc, flags, window):
    R, d = 3, 12
    inp, ps = _bps("halton", R, d, flags=flags, seed=10 + flags)
    got = ldk.gen_bpoints(ps, *window).cpu().numpy()
    ref = orc.bpoints("halton", R, d, *window, flags=flags, **inp)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("flags", FLAG_SETS)
@pytest.mark.parametrize("b,d", [(13, 10), (2, 2), (53, 52)])
def test_faure_bit_exact(orc, flags, b, d):
    R = 2
    n = 2000 if d < 52 else 600
    inp, ps = _bps("faure", R, d, base=b, flags=flags, seed=20 + flags)
    got = ldk.gen_bpoints(ps, 5, 5 + n).cpu().numpy()
    ref = orc.bpoints("faure", R, d, 5, 5 + n, base=b, flags=flags, **inp)
    assert np.array_equal(got, ref)


def test_halton_largest_dimension_and_large_index(orc):
    # 54 dimensions (bases up to 251), indices past 2^20 (more index digits)
    R, d = 2, 54
    inp, ps = _bps("halton", R, d, flags=7, seed=5)
    lo, hi = 2**20 - 300, 2**20 + 300
    got = ldk.gen_bpoints(ps, lo, hi).cpu().numpy()
    assert np.array_equal(got, orc.bpoints("halton", R, d, lo, hi, flags=7, **inp))


@pytest.mark.parametrize("flags", [0, 7])
@pytest.mark.parametrize("kind,base,d", [("halton", 0, 8), ("faure", 3, 3), ("faure", 251, 3)])
def test_indices_below_two_to_32(orc, kind, base, d, flags):
    # the top of the index range: 32 base-2 digits (the longest packed digit
    # vector), 21 base-3 digits, 5 base-251 digits; the 32-bit division at
    # its largest arguments
    R = 2
    inp, ps = _bps(kind, R, d, base=base, flags=flags, seed=41)
    lo, hi = 2**32 - 700, 2**32
    got = ldk.gen_bpoints(ps, lo, hi).cpu().numpy()
    assert np.array_equal(got, orc.bpoints(kind, R, d, lo, hi, base=base, flags=flags, **inp))


@pytest.mark.parametrize("b,d", [(61, 60), (97, 90)])
def test_faure_more_dimensions_than_halton(orc, b, d):
    # Faure allows d up to its base (251): more dimensions than the Halton
    # bases, every one sharing the base
    R = 2
    inp, ps = _bps("faure", R, d, base=b, flags=7, seed=43)
    got = ldk.gen_bpoints(ps, 11, 320).cpu().numpy()
    assert np.array_equal(got, orc.bpoints("faure", R, d, 11, 320, base=b, flags=7, **inp))


@pytest.mark.parametrize("d", [1, 5, 70])
@pytest.mark.parametrize("window", [(0, 4096), (100, 3001)])
def test_nus_bit_exact(orc, window, d):
    # d = 70: two output tiles of dimensions
    m, R = 12, 3
    t = W.small_net(8, m, d, R)
    seed = W.nus_seeds(8, R, d)
    ps = ldk.BPointSet("nus", R, d, gen=dev_u64(t["gen"]), seed=dev_u64(seed), m=m)
    got = ldk.gen_bpoints(ps, *window).cpu().numpy()
    ref = orc.unit_points(orc.nus_points(t["gen"], seed, m, *window))
    assert np.array_equal(got, ref)


def test_empty_window_and_argument_errors():
    inp, ps = _bps("halton", 1, 4, flags=7)
    out = torch.full((1, 0, 4), 7.0, dtype=torch.float64, device="cuda")
    ldk.gen_bpoints(ps, 9, 9, out=out)
    with pytest.raises(ldk.LdkError):
        ldk.gen_bpoints(ldk.BPointSet("halton", 1, 55), 0, 8)  # more dimensions than bases
    with pytest.raises(ldk.LdkError):
        ldk.gen_bpoints(ldk.BPointSet("faure", 1, 4, base=9), 0, 8)  # not prime
    with pytest.raises(ldk.LdkError):
        ldk.gen_bpoints(ldk.BPointSet("faure", 1, 6, base=5), 0, 8)  # base below d
    with pytest.raises(ldk.LdkError):
        ldk.gen_bpoints(ldk.BPointSet("halton", 1, 4, flags=ldk.BR_LMS), 0, 8)  # no S
    t = W.small_net(1, 4, 2, 1)
    nus = ldk.BPointSet("nus", 1, 2, gen=dev_u64(t["gen"]),
                        seed=dev_u64(W.nus_seeds(1, 1, 2)), m=4)
    with pytest.raises(ldk.LdkError):
        ldk.gen_bpoints(nus, 0, 17)  # beyond 2^m


@pytest.mark.parametrize("integrand", ["corner_peak", "oscillatory"])
@pytest.mark.parametrize("kind", ["halton", "faure", "nus"])
def test_rqmc_over_points_matches_oracle(orc, integrand, kind):
    from test_gpu_rqmc import _check
    R, d, n = 8, 20, 3000
    c = W.corner_peak_coefficients(d)
    if kind == "nus":
        m = 12
        t = W.small_net(9, m, d, R)
        seed = W.nus_seeds(9, R, d)
        ps = ldk.BPointSet("nus", R, d, gen=dev_u64(t["gen"]), seed=dev_u64(seed), m=m)
        xh = orc.unit_points(orc.nus_points(t["gen"], seed, m, 0, n))
    else:
        base = 23 if kind == "faure" else 0
        inp, ps = _bps(kind, R, d, base=base, flags=1 | 2, seed=9)
        xh = orc.bpoints(kind, R, d, 0, n, base=base, flags=1 | 2, **inp)
    x = ldk.gen_bpoints(ps, 0, n)
    assert np.array_equal(x.cpu().numpy(), xh)
    y = orc.genz_corner_peak(xh, c) if integrand == "corner_peak" else \
        orc.genz_oscillatory(xh, c, 0.3)
    ref = orc.rqmc(y, tau=0.01)
    mu_r, stats = ldk.rqmc_points(x, integrand, torch.from_numpy(c).cuda(), u=0.3, tau=0.01)
    _check(f"rqmc_points_{kind}_{integrand}", mu_r.cpu().numpy(), stats.cpu().numpy(), ref, y,
           integrand, c, n)


@pytest.mark.parametrize("integrand", ["corner_peak", "oscillatory"])
@pytest.mark.parametrize("R,n,d", [(1, 1, 1), (3, 255, 17), (2, 257, 52), (4, 5000, 52), (2, 700, 128),
                                   (2, 4099, 16)])
def test_rqmc_points_shapes(orc, integrand, R, n, d):
    # any coordinates in [0, 1): ragged tiles (n not a multiple of 256 points),
    # d from 1 to the largest (128), one replication (no interval)
    from test_gpu_rqmc import _check
    rng = np.random.default_rng(1000 * d + n)
    xh = rng.random((R, n, d))
    c = W.corner_peak_coefficients(d)
    y = orc.genz_corner_peak(xh, c) if integrand == "corner_peak" else orc.genz_oscillatory(xh, c, 0.3)
    ref = orc.rqmc(y, tau=0.01)
    mu_r, stats = ldk.rqmc_points(torch.from_numpy(xh).cuda(), integrand, torch.from_numpy(c).cuda(), u=0.3,
                                  tau=0.01)
    _check(f"rqmc_points_R{R}_n{n}_d{d}_{integrand}", mu_r.cpu().numpy(), stats.cpu().numpy(), ref, y,
           integrand, c, n)


@pytest.mark.parametrize("kind,base", [("halton", 0), ("faure", 53), ("nus", 0)])
def test_bench_shape_sampled(orc, kind, base):
    # the benchmark's shape and launch (R = 16, d = 52, the whole window
    # [0, 2^16) in one call, LMS + digit permutations for Halton and Faure),
    # rows sampled at the start, across a tile boundary and at the end, each
    # bit for bit against the oracle's window
    R, d, m = 16, 52, 16
    n = 2**m
    if kind == "nus":
        t = W.small_net(31, m, d, 1)
        seed = W.nus_seeds(31, R, d)
        ps = ldk.BPointSet("nus", R, d, m=m, gen=dev_u64(t["gen"]), seed=dev_u64(seed))
    else:
        inp, ps = _bps(kind, R, d, base=base, flags=ldk.BR_LMS | ldk.BR_DP, seed=31)
    x = ldk.gen_bpoints(ps, 0, n).cpu().numpy()
    for lo, hi in ((0, 70), (4070, 4170), (n - 90, n)):
        if kind == "nus":
            ref = orc.unit_points(orc.nus_points(t["gen"], seed, m, lo, hi))
        else:
            ref = orc.bpoints(kind, R, d, lo, hi, base=base, flags=ldk.BR_LMS | ldk.BR_DP, **inp)
        assert np.array_equal(x[:, lo:hi], ref), (lo, hi)


def test_rqmc_points_bench_shape(orc):
    # the benchmark's RQMC-over-points shape and launch (R = 16, n = 2^16,
    # d = 52, 436 MB of coordinates), seeded coordinates in [0, 1)
    from test_gpu_rqmc import _check
    R, n, d = 16, 2**16, 52
    xh = np.random.default_rng(52).random((R, n, d))
    c = W.corner_peak_coefficients(d)
    y = orc.genz_corner_peak(xh, c)
    ref = orc.rqmc(y, tau=0.01)
    mu_r, stats = ldk.rqmc_points(torch.from_numpy(xh).cuda(), "corner_peak", torch.from_numpy(c).cuda(),
                                  tau=0.01)
    _check("rqmc_points_bench_shape", mu_r.cpu().numpy(), stats.cpu().numpy(), ref, y, "corner_peak", c, n)
