"""Pins for the oracle's point generators (Sec. 4.1-4.3), CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import brute
from golden_io import rows


def test_gray_code_matches_table1(orc):
    # Table 1, base 2, rows 0..7 (row 8 is a misprint; see the fixture header)
    for i, ib, gb in rows("gray_code_b2.txt"):
        i = int(i)
        assert int(ib, 2) == i
        assert orc.gray(i) == int(gb, 2)
    # the rule stated in the text: consecutive codes differ in exactly one digit
    for i in range(4096):
        assert bin(orc.gray(i) ^ orc.gray(i + 1)).count("1") == 1
    assert orc.gray(8) == 0b1100


def _unpack_cols(cols, m):
    # 64 x m 0/1 matrix, row t = bit 63 - t
    return np.array([[(int(cols[k]) >> (63 - t)) & 1 for k in range(m)] for t in range(64)])


def _unpack_rows(rws):
    return np.array([[(int(rws[t]) >> (63 - s)) & 1 for s in range(64)] for t in range(64)])


def _pack_digits(z):
    u = 0
    for t in range(64):
        if z[t] & 1:
            u |= 1 << (63 - t)
    return u


@pytest.mark.parametrize("order", ["natural", "gray"])
def test_dnet_matches_dense_gf2_definition(orc, order):
    # Sec. 4.3: z = F(S C D_m(i) mod 2), x = z (+) Delta, brute force on 0/1 digits
    w = W.small_net(11, m=5, d=3, R=2)
    pts = orc.points(w, order=order)
    for r in range(w["R"]):
        for j in range(w["d"]):
            Cm = _unpack_cols(w["gen"][j], w["m"])
            Sm = _unpack_rows(w["lms"][r, j])
            Ct = (Sm @ Cm) % 2
            delta = [(int(w["shift"][r, j]) >> (63 - t)) & 1 for t in range(64)]
            for i in range(2 ** w["m"]):
                code = i ^ (i >> 1) if order == "gray" else i
                dvec = np.array([(code >> k) & 1 for k in range(w["m"])])
                z = (Ct @ dvec) % 2
                x = [(int(z[t]) + delta[t]) % 2 for t in range(64)]
                assert int(pts[r, i, j]) == _pack_digits(x)


def test_dnet_identity_is_van_der_corput(orc):
    m = 8
    C = np.array([[1 << (63 - k) for k in range(m)]], dtype=np.uint64)
    pts = orc.dnet_points(C, None, None, m, 0, 2**m, R=1)
    for i in range(2**m):
        # v(i) = sum_t i_{t-1} 2^-t, digit t at bit 64 - t
        v = sum(((i >> (t - 1)) & 1) << (64 - t) for t in range(1, m + 1))
        assert int(pts[0, i, 0]) == v


def test_dnet_stratification_and_gray_permutation(orc):
    w = W.workload(1)
    m = w["m"]
    nat = orc.points(w)
    gry = orc.points(w, order="gray")
    for j in range(w["d"]):
        top = (nat[0, :, j] ^ w["shift"][0, j]) >> np.uint64(64 - m)
        assert sorted(top.tolist()) == list(range(2**m))
    # Gray order lists the same set; point i is the natural point gray(i)
    idx = np.array([orc.gray(i) for i in range(2**m)])
    assert np.array_equal(gry[0], nat[0, idx])
    # one column per step: x_{i+1} (+) x_i = Ct[:, ctz(i+1)]
    Ct = orc.lms(w["gen"], w["lms"][0])
    for i in range(2**m - 1):
        q = ((i + 1) & -(i + 1)).bit_length() - 1
        assert np.array_equal(gry[0, i + 1] ^ gry[0, i], Ct[:, q])


def test_point_windows_match_full(orc):
    w = W.small_net(5, m=7, d=4, R=2)
    full = orc.points(w)
    assert np.array_equal(orc.points(w, 37, 101), full[:, 37:101])
    wl = W.small_lattice(6, m=7, d=4, R=2)
    full = orc.points(wl)
    assert np.array_equal(orc.points(wl, 3, 90), full[:, 3:90])


def test_lattice_natural_equals_linear_via_bit_reversal(orc):
    # Sec. 4.2: v(i) g mod 1 = R_m(i) g / n mod 1 for i < 2^m, so the natural
    # and linear point sets coincide at n = 2^m
    for m in (0, 1, 5, 10):
        w = W.small_lattice(20 + m, m=m, d=3, R=1)
        nat = orc.points(w)
        lin = orc.points(w, order="linear")
        for i in range(2**m):
            assert np.array_equal(nat[0, i], lin[0, brute.bitrev(i, m)])
        assert sorted(map(tuple, nat[0].tolist())) == sorted(map(tuple, lin[0].tolist()))


def test_lattice_linear_is_ign(orc):
    # linear order: (x_i - Delta) mod 1 = frac(i g / n), exact in integers
    w = W.small_lattice(3, m=9, d=5, R=2)
    lin = orc.points(w, order="linear")
    n = 2 ** w["m"]
    for r in range(2):
        for i in range(0, n, 7):
            for j in range(5):
                u = (int(lin[r, i, j]) - int(w["shift"][r, j])) % 2**64
                assert u == ((i * int(w["gen"][j])) % n) * 2 ** (64 - w["m"])


def test_lattice_g1_is_van_der_corput(orc):
    pts = orc.lattice_points(np.array([1], dtype=np.uint64), None, 10, 0, 1024)
    for i in range(1024):
        assert int(pts[0, i, 0]) == brute.bitrev(i, 64)
