"""Pins for the oracle's transforms (Figure 3, Sec. 5.2-5.4), CPU only."""
import numpy as np
import pytest

from oracle import brute


@pytest.mark.parametrize("m", range(0, 9))
def test_fwht_is_normalised_hadamard(orc, m):
    rng = np.random.default_rng(m)
    x = rng.standard_normal(2**m)
    H = brute.hadamard(m)
    np.testing.assert_allclose(orc.fwht(x), H @ x / np.sqrt(2**m), rtol=0, atol=1e-13)
    # FWHT applied twice is the identity; unnormalised H_m H_m = n I
    np.testing.assert_allclose(orc.fwht(orc.fwht(x)), x, rtol=0, atol=1e-13)
    np.testing.assert_array_equal(H @ H, (2**m) * np.eye(2**m))


@pytest.mark.parametrize("m", range(0, 9))
def test_fftbr_is_bit_reversed_dft(orc, m):
    rng = np.random.default_rng(10 + m)
    n = 2**m
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    # direct matrix W^{k R_m(j)}
    np.testing.assert_allclose(orc.fftbr(x), brute.fourier_br(m) @ x / np.sqrt(n), atol=1e-13)
    # numpy's FFT of the linear-order sequence x_lin[R(j)] = x[j]
    lin = np.empty_like(x)
    for j in range(n):
        lin[brute.bitrev(j, m)] = x[j]
    np.testing.assert_allclose(orc.fftbr(x), np.fft.fft(lin) / np.sqrt(n), atol=1e-13)
    # IFFTBR is the inverse and the conjugate transpose
    np.testing.assert_allclose(orc.ifftbr(orc.fftbr(x)), x, atol=1e-13)
    np.testing.assert_allclose(orc.ifftbr(x), brute.fourier_br(m).conj().T @ x / np.sqrt(n),
                               atol=1e-13)


def test_batched_transform_matches_rows(orc):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 64)) + 1j * rng.standard_normal((3, 64))
    out = orc.transform("lattice", x)
    for b in range(3):
        np.testing.assert_allclose(out[b], orc.fftbr(x[b]), atol=0, rtol=0)
    back = orc.transform("lattice", out, inverse=True)
    np.testing.assert_allclose(back, x, atol=1e-13)
    xr = rng.standard_normal((3, 64))
    outr = orc.transform("dnet", xr)
    for b in range(3):
        np.testing.assert_array_equal(outr[b], orc.fwht(xr[b]))
    # long-double twin agrees to FP64 rounding
    np.testing.assert_allclose(orc.transform("lattice", x, precise=True), out, atol=1e-14)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
@pytest.mark.parametrize("m", [0, 1, 3, 7])
def test_update_double_equals_fresh_transform(orc, kind, m):
    # Sec. 5.4 / eq. (ft_next_parts): reuse the size-n transform when n doubles
    rng = np.random.default_rng(m)
    n = 2**m
    y = rng.standard_normal((2, n))
    ynew = rng.standard_normal((2, n))
    if kind == "lattice":
        yt = orc.transform(kind, y.astype(np.complex128))
        fresh = orc.transform(kind, np.concatenate([y, ynew], axis=1).astype(np.complex128))
    else:
        yt = orc.transform(kind, y)
        fresh = orc.transform(kind, np.concatenate([y, ynew], axis=1))
    np.testing.assert_allclose(orc.update_double(kind, yt, ynew), fresh, atol=1e-13)


@pytest.mark.parametrize("kind", ["lattice", "dnet"])
def test_eig_update_double_equals_fresh_eig(orc, kind):
    rng = np.random.default_rng(4)
    n = 32
    # a symmetric first column is needed only for real lattice spectra of the
    # full size; use an actual lattice / net column
    import workloads as W

    w = (W.small_lattice(8, m=6, d=3) if kind == "lattice" else W.small_net(8, m=6, d=3))
    w.update(alpha=np.full(3, 2, np.int32), gamma=np.array([1.0, 0.5, 0.25]), zeta=1.0)
    pts = orc.points(w)
    k1 = orc.kernel_column(kind, pts, pts[:, 0, :], w["alpha"], w["gamma"], 1.0)
    lam_half, _ = orc.eig(kind, k1[:, :n])
    lam_full, _ = orc.eig(kind, k1)
    upd = orc.eig_update_double(kind, lam_half, k1[:, n:])
    np.testing.assert_allclose(upd, lam_full, atol=1e-12 * np.abs(lam_full).max())
    assert rng is not None
