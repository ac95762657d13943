"""Pins of the oracle's point sets without FWHT structure (Secs. 4.3 and 4.4):
Halton and Faure points with LMS, digit permutations and digital shifts, and
nested uniform scrambling of a base-2 net.

What fixes them:
- Halton, unrandomized: the radical inverse of i in the j-th prime base, as
  an exact rational (Python fractions), rounded once.
- Faure, unrandomized: Faure's sequence in base b >= s is a (0, s)-sequence,
  so the first b^m points are a (0, m, s)-net: every elementary interval
  prod_j [a_j b^-k_j, (a_j + 1) b^-k_j) with sum k_j = m holds exactly one
  point (brute force); its first dimension is the van der Corput sequence.
  LMS by a nonsingular lower-triangular S keeps the net property, and so
  does a digital shift.
- DS and DP: undoing the shift (digit-wise, mod b) or the permutations
  digit by digit gives the unrandomized digits; LMS gives S z mod b of the
  unrandomized digit vector (brute force on the digits).
- NUS: digit t of a scrambled coordinate depends only on the unscrambled
  digits 1..t, each level is a bijection of {0, 1} (so two points first
  differing at digit p still differ there, and agree before it), the net's
  stratification survives, and the flips are balanced.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def digits_of(x, b, T):
    """The T base-b digits (most significant first) of the coordinates x, from
    the exact rational value of each double: x b^T is within 1/2 of the
    integer v = sum_t z_t b^(T-1-t) because b^T <= 2^53."""
    out = np.empty(x.shape + (T,), np.int64)
    bT = b**T
    for idx in np.ndindex(x.shape):
        v = round(Fraction(float(x[idx])) * bT)
        for t in range(T - 1, -1, -1):
            out[idx + (t,)] = v % b
            v //= b
    return out


def test_digit_counts_and_primes():
    for b in (2, 3, 5, 7, 239, 251):
        T = oracle.bdigits(b)
        assert b**T <= 2**53 < b ** (T + 1)
    primes = [p for p in range(2, 300) if all(p % q for q in range(2, int(p**0.5) + 1))]
    assert [oracle.nth_prime(j) for j in range(1, 55)] == primes[:54]


def test_halton_is_the_radical_inverse():
    d, n = 12, 300
    x = oracle.bpoints("halton", 1, d, 0, n)[0]
    for j in range(d):
        b = oracle.nth_prime(j + 1)
        for i in range(n):
            v, f, k = Fraction(0), Fraction(1, b), i
            while k:
                v += (k % b) * f
                k //= b
                f /= b
            assert x[i, j] == float(v), (i, j)
    # a window starting past zero is the same rows
    assert np.array_equal(oracle.bpoints("halton", 1, d, 37, 123)[0], x[37:123])


def _elementary_ok(x, b, m):
    """Every elementary interval of volume b^-m holds exactly one of the b^m
    points.  The cell index comes from the exact digit integer v of each
    coordinate (a double's floor(x b^k) can fall one short on a boundary)."""
    n, s = x.shape
    assert n == b**m
    T = oracle.bdigits(b)
    v = [[round(Fraction(float(x[i, j])) * b**T) for j in range(s)] for i in range(n)]
    for ks in itertools.product(range(m + 1), repeat=s):
        if sum(ks) != m:
            continue
        cells = set()
        for i in range(n):
            cells.add(tuple(v[i][j] // b ** (T - ks[j]) for j in range(s)))
        if len(cells) != n:
            return False
    return True


@pytest.mark.parametrize("b,s,m", [(2, 2, 4), (3, 3, 3), (5, 5, 2), (5, 4, 3), (7, 3, 2)])
def test_faure_is_a_zero_m_s_net(b, s, m):
    x = oracle.bpoints("faure", 1, s, 0, b**m, base=b)[0]
    assert _elementary_ok(x, b, m)
    # the first dimension is van der Corput in base b
    for i in range(b**m):
        v, f, k = Fraction(0), Fraction(1, b), i
        while k:
            v += (k % b) * f
            k //= b
            f /= b
        assert x[i, 0] == float(v)


def test_faure_net_property_fails_for_a_wrong_matrix():
    # the brute-force check has teeth: dimension pairs of the Halton set
    # (different bases) or a repeated Faure dimension are not (0, m, 2)-nets
    x = oracle.bpoints("faure", 1, 3, 0, 27, base=3)[0]
    rep = np.stack([x[:, 1], x[:, 1], x[:, 2]], axis=1)
    assert not _elementary_ok(rep, 3, 3)


@pytest.mark.parametrize("flags", [1, 4, 1 | 4])
def test_faure_randomized_keeps_the_net_property(flags):
    b, s, m = 5, 4, 3
    inp = W.bpoint_inputs(7, "faure", 2, s, base=b)
    x = oracle.bpoints("faure", 2, s, 0, b**m, base=b, flags=flags, **inp)
    for r in range(2):
        assert _elementary_ok(x[r], b, m)


@pytest.mark.parametrize("kind,base", [("halton", 0), ("faure", 7)])
def test_randomizations_undo_to_the_plain_digits(kind, base):
    R, d, n = 2, 5, 60
    inp = W.bpoint_inputs(11, kind, R, d, base=base)
    plain = oracle.bpoints(kind, R, d, 0, n, base=base)
    for j in range(d):
        b = base if kind == "faure" else oracle.nth_prime(j + 1)
        T = oracle.bdigits(b)
        zp = digits_of(plain[:, :, j], b, T)  # [R][n][T]
        # DS alone
        xs = oracle.bpoints(kind, R, d, 0, n, base=base, flags=oracle.BR_DS, **inp)
        zs = digits_of(xs[:, :, j], b, T)
        sh = inp["shift"][:, j, :T].astype(np.int64)[:, None, :]
        assert np.array_equal((zs - sh) % b, zp)
        # DP alone
        xp = oracle.bpoints(kind, R, d, 0, n, base=base, flags=oracle.BR_DP, **inp)
        zq = digits_of(xp[:, :, j], b, T)
        for r in range(R):
            inv = np.empty((T, b), np.int64)
            for t in range(T):
                pi = inp["perm"][r, j, t, :b].astype(np.int64)
                assert sorted(pi.tolist()) == list(range(b))
                inv[t, pi] = np.arange(b)
            assert np.array_equal(inv[np.arange(T)[None, :], zq[r]], zp[r])
        # LMS alone: S z mod b of the plain digit vector
        xl = oracle.bpoints(kind, R, d, 0, n, base=base, flags=oracle.BR_LMS, **inp)
        zl = digits_of(xl[:, :, j], b, T)
        for r in range(R):
            S = inp["lms"][r, j, :T, :T].astype(np.int64)
            assert np.all(np.triu(S, 1) == 0) and np.all(np.diag(S) % b != 0)
            assert np.array_equal((zp[r] @ S.T) % b, zl[r])
        # all three, in the order LMS, DP, DS
        xa = oracle.bpoints(kind, R, d, 0, n, base=base, flags=7, **inp)
        za = digits_of(xa[:, :, j], b, T)
        for r in range(R):
            S = inp["lms"][r, j, :T, :T].astype(np.int64)
            z = (zp[r] @ S.T) % b
            z = np.stack([inp["perm"][r, j, t, :][z[:, t]] for t in range(T)], axis=1)
            z = (z + inp["shift"][r, j, :T]) % b
            assert np.array_equal(za[r], z)


def _bits(words):
    w = np.asarray(words, np.uint64)
    return ((w[..., None] >> np.arange(63, -1, -1, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)


def test_nus_prefix_structure_and_bijection():
    m, d, R = 10, 3, 2
    t = W.small_net(5, m, d, R)
    seed = W.nus_seeds(5, R, d)
    z = oracle.dnet_points(t["gen"], None, None, m, 0, 2**m)  # unscrambled words [1][n][d]
    x = oracle.nus_points(t["gen"], seed, m, 0, 2**m)
    zb, xb = _bits(z[0]), _bits(x)
    rng = np.random.default_rng(0)
    for _ in range(400):
        i, k = rng.integers(0, 2**m, 2)
        for r in range(R):
            for j in range(d):
                a, b = zb[i, j], zb[k, j]
                diff = np.nonzero(a != b)[0]
                p = diff[0] if diff.size else 64
                # agree before the first differing digit, differ at it
                assert np.array_equal(xb[r, i, j, :p], xb[r, k, j, :p])
                if p < 64:
                    assert xb[r, i, j, p] != xb[r, k, j, p]
    # the first digit is flipped for every point or for none (empty prefix)
    for r in range(R):
        for j in range(d):
            f = xb[r, :, j, 0] ^ zb[:, j, 0]
            assert np.all(f == f[0])
    # different seeds give different scrambles
    assert not np.array_equal(x[0], x[1])


def test_nus_keeps_the_stratification():
    # identity generating columns: van der Corput; after NUS the first 2^m
    # points still fall one per interval [a 2^-m, (a + 1) 2^-m)
    m = 9
    C_ = np.array([[np.uint64(1) << np.uint64(63 - k) for k in range(m)]], np.uint64)
    seed = W.nus_seeds(9, 3, 1)
    x = oracle.nus_points(C_, seed, m, 0, 2**m)
    for r in range(3):
        cells = (x[r, :, 0] >> np.uint64(64 - m)).astype(np.int64)
        assert sorted(cells.tolist()) == list(range(2**m))


def test_nus_flips_are_balanced():
    # level-t flips over the 2^(t-1) prefixes of a full net are about half
    # ones: the generator's top bit is unbiased (binomial, 6 sigma)
    m = 12
    C_ = np.array([[np.uint64(1) << np.uint64(63 - k) for k in range(m)]], np.uint64)
    seed = W.nus_seeds(3, 1, 1)
    z = oracle.dnet_points(C_, None, None, m, 0, 2**m)[0, :, 0]
    x = oracle.nus_points(C_, seed, m, 0, 2**m)[0, :, 0]
    flips = _bits(x ^ z)
    zb = _bits(z)
    for t in range(4, m):
        # one flip per distinct prefix of length t
        pre = {}
        for i in range(2**m):
            pre[tuple(zb[i, :t])] = flips[i, t]
        k = len(pre)
        ones = sum(pre.values())
        assert abs(ones - k / 2) <= 6 * math.sqrt(k / 4) + 1, (t, ones, k)
    # the mixing function spreads a one-bit change of its input (avalanche)
    rng = np.random.default_rng(1)
    tot = 0
    for _ in range(200):
        v = int(rng.integers(0, 2**63)) * 2 + 1
        for bit in (0, 17, 40, 63):
            tot += bin(oracle.mix64(v) ^ oracle.mix64(v ^ (1 << bit))).count("1")
    assert abs(tot / 800 - 32) < 2
