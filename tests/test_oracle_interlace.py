"""Oracle pins for digital interlacing and higher-order LMS nets (Sec. 4.3):
the printed interlacing example, the identity at alpha = 1, and the
interlaced net's points against the digit-interlaced points of the
alpha d-dimensional net (the net is linear in its generating matrices, so
interlacing the matrices interlaces the points' digits)."""
import numpy as np
import pytest

import workloads as W
from golden_io import rows


def _bit(t):
    return np.uint64(1) << np.uint64(63 - t)


def test_interlace_matches_printed_example(orc):
    # m = 2, t_max = 2, alpha = 2, four source matrices: place a single 1 at
    # every source entry (j, t, k) in turn and find where interlacing moves it
    where = {}
    for jh, th, k, j, t in rows("interlace_example_b2.txt"):
        where[(int(j), int(t), int(k))] = (int(jh), int(th), int(k))
    assert len(where) == 16
    for (j, t, k), (jh, th, kh) in where.items():
        cols = np.zeros((4, 2), np.uint64)
        cols[j - 1, k - 1] = _bit(t)
        out = orc.interlace(cols, 2)
        want = np.zeros((2, 2), np.uint64)
        want[jh - 1, kh - 1] = _bit(th)
        assert np.array_equal(out, want), (j, t, k)


def test_interlace_alpha_one_is_identity(orc):
    rng = np.random.default_rng(4)
    cols = rng.integers(0, 2**63, size=(5, 7), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    assert np.array_equal(orc.interlace(cols, 1), cols)


def _digit_interlace(P, alpha):
    """Digit t of coordinate j = digit t // alpha of coordinate alpha j + t % alpha."""
    n, ad = P.shape
    d = ad // alpha
    out = np.zeros((n, d), np.uint64)
    for j in range(d):
        for t in range(64):
            src = P[:, alpha * j + t % alpha]
            bit = (src >> np.uint64(63 - t // alpha)) & np.uint64(1)
            out[:, j] |= bit << np.uint64(63 - t)
    return out


@pytest.mark.parametrize("alpha", [2, 3, 4])
@pytest.mark.parametrize("order", ["natural", "gray"])
def test_interlaced_net_points_are_interlaced_digits(orc, alpha, order):
    m, d, R = 7, 3, 2
    w = W.small_net(40 + alpha, m=m, d=alpha * d, R=R)
    n = 2**m
    pts = orc.higher_order_dnet_points(w["gen"], w["lms"], None, alpha, m, 0, n, order)
    for r in range(R):
        # the alpha d-dimensional net of replication r's scrambled matrices
        src = orc.dnet_points(w["gen"], w["lms"][r:r + 1], None, m, 0, n, order, R=1)[0]
        assert np.array_equal(pts[r], _digit_interlace(src, alpha)), r


def test_higher_order_net_shift_is_applied_after_interlacing(orc):
    alpha, m, d = 2, 5, 2
    w = W.small_net(9, m=m, d=alpha * d, R=1)
    shift = np.array([[0x8000000000000001, 0x0123456789ABCDEF]], np.uint64)
    plain = orc.higher_order_dnet_points(w["gen"], w["lms"], None, alpha, m, 0, 2**m)
    shifted = orc.higher_order_dnet_points(w["gen"], w["lms"], shift, alpha, m, 0, 2**m)
    assert np.array_equal(shifted, plain ^ shift[:, None, :])
