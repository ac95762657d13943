"""Seeded synthetic inputs for the fast kernel-method path.

This module is shared by the oracle-side tests and the GPU-side tests and
benchmark.  It only draws random numbers and lays them out; it holds none of
the method's arithmetic (no point generation, no kernel, no transform).

Layouts (all little-endian, row-major):

* lattice generating vector ``g``: ``uint64[d]``, odd, ``< 2**m_max``
  (Sec. 4.2: rank-1 lattice with generating vector g).
* digital-net generating matrices ``C``: ``uint64[d][m_max]``, one word per
  column k; the digit of weight ``2**-(t+1)`` (row t) is bit ``63 - t``
  (Sec. 4.3: generating matrices C_j in {0,1}^{t_max x m}, t_max = 64).
* linear matrix scrambling ``S``: ``uint64[R][d][64]``, one word per row t;
  entry (t, s) is bit ``63 - s``; unit lower-triangular (Matousek, Sec. 4.3).
* shifts: ``uint64[R][d]``; a digital shift's digit t is bit ``63 - t``; a
  lattice shift is the 64-bit fixed-point value ``Delta * 2**64``.

The five named workloads follow the shapes of the fast-kernel experiments:
the seed of ``workload(k)`` is ``k``; draw order is generating vector or
matrices, then S, then shifts, then responses, looping over replications or
instances in index order.
"""
from __future__ import annotations

import math

import numpy as np

U64 = np.uint64


def _u64(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.integers(0, 2**64, size=shape, dtype=np.uint64, endpoint=False)


def lattice_generating_vector(rng: np.random.Generator, d: int, m: int) -> np.ndarray:
    """Random odd integers in [1, 2**m): g_j = 2*U{0..2**(m-1)-1} + 1."""
    if m == 0:
        return np.ones(d, dtype=np.uint64)
    half = rng.integers(0, 2 ** (m - 1), size=d, dtype=np.uint64)
    return (half * U64(2) + U64(1)).astype(np.uint64)


def net_generating_matrices(rng: np.random.Generator, d: int, m: int) -> np.ndarray:
    """Random 64 x m matrices, unit upper-triangular in their top m rows.

    Rows 0..m-1 form a unit upper-triangular m x m block (random bits above
    the diagonal, zeros below); rows m..63 are random bits.  Returned as
    ``uint64[d][m]`` columns with row t at bit 63 - t.
    """
    cols = np.zeros((d, m), dtype=np.uint64)
    for j in range(d):
        for k in range(m):
            w = int(_u64(rng, 1)[0])
            # keep rows t < k (bits 63..64-k) random, set row k, clear rows k+1..m-1,
            # keep rows >= m random
            keep_top = ((1 << k) - 1) << (64 - k) if k > 0 else 0
            keep_low = (1 << (64 - m)) - 1 if m < 64 else 0
            w = (w & (keep_top | keep_low)) | (1 << (63 - k))
            cols[j, k] = w
    return cols


def lms_matrices(rng: np.random.Generator, R: int, d: int) -> np.ndarray:
    """Unit lower-triangular 64 x 64 scrambles (Matousek), ``uint64[R][d][64]`` rows."""
    out = np.zeros((R, d, 64), dtype=np.uint64)
    for r in range(R):
        for j in range(d):
            words = _u64(rng, 64)
            for t in range(64):
                below = ((1 << t) - 1) << (64 - t) if t > 0 else 0  # columns s < t
                out[r, j, t] = (int(words[t]) & below) | (1 << (63 - t))
    return out


def shifts(rng: np.random.Generator, R: int, d: int) -> np.ndarray:
    """Uniform 64-bit shifts ``uint64[R][d]`` (digital or fixed-point)."""
    return _u64(rng, (R, d))


def to_unit_f64(u: np.ndarray) -> np.ndarray:
    """Float view of 64-bit fixed-point coordinates: (u >> 11) * 2**-53 (exact)."""
    return (np.asarray(u, dtype=np.uint64) >> U64(11)).astype(np.float64) * 2.0**-53


def sine_response(x: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """y = sum_j sin(2 pi x_j) / j + eps for points x of shape (..., n, d)."""
    d = x.shape[-1]
    w = 1.0 / np.arange(1, d + 1, dtype=np.float64)
    return np.sin(2.0 * math.pi * x) @ w + eps


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def workload(k: int) -> dict:
    """The five workloads: 1 parity net, 2 lattice n=2^20, 3 net n=2^20,
    4 batched mixed instances, 5 marginal-likelihood gradient."""
    return {1: _w1, 2: _w2, 3: _w3, 4: _w4, 5: _w5}[k]()


def _w1() -> dict:
    rng = np.random.default_rng(1)
    m, d, R = 10, 4, 1
    C = net_generating_matrices(rng, d, m)
    S = lms_matrices(rng, R, d)
    D = shifts(rng, R, d)
    y = rng.standard_normal((R, 1, 2**m))
    return dict(name="net_m10_d4_dsi1", kind="dnet", order="natural", m=m, d=d, R=R,
                gen=C, lms=S, shift=D, alpha=np.full(d, 1, np.int32),
                gamma=np.ones(d), zeta=1.0, sigma2=1e-8, y=y, nrhs=1)


def _w2() -> dict:
    rng = np.random.default_rng(2)
    m, d, R = 20, 32, 1
    g = lattice_generating_vector(rng, d, m)
    D = shifts(rng, R, d)
    eps = rng.normal(0.0, math.sqrt(1e-3), size=(R, 1, 2**m))
    return dict(name="lattice_m20_d32_si2", kind="lattice", order="natural", m=m, d=d, R=R,
                gen=g, lms=None, shift=D, alpha=np.full(d, 2, np.int32),
                gamma=1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2, zeta=1.0,
                sigma2=1e-3, eps=eps, nrhs=1)


def _w3() -> dict:
    rng = np.random.default_rng(3)
    m, d, R = 20, 32, 1
    C = net_generating_matrices(rng, d, m)
    S = lms_matrices(rng, R, d)
    D = shifts(rng, R, d)
    y = rng.standard_normal((R, 1, 2**m))
    return dict(name="net_m20_d32_dsi4", kind="dnet", order="natural", m=m, d=d, R=R,
                gen=C, lms=S, shift=D, alpha=np.full(d, 4, np.int32),
                gamma=0.5 ** np.arange(1, d + 1, dtype=np.float64), zeta=1.0,
                sigma2=1e-8, y=y, nrhs=1)


def _w4() -> dict:
    rng = np.random.default_rng(4)
    n_inst, d, nrhs, mmax = 256, 16, 8, 18
    m_r = rng.integers(12, 19, size=n_inst)
    kinds = rng.integers(0, 2, size=n_inst)  # 0 lattice, 1 net
    g = lattice_generating_vector(rng, d, mmax)
    C = net_generating_matrices(rng, d, mmax)
    inst = []
    for r in range(n_inst):
        S = lms_matrices(rng, 1, d) if kinds[r] == 1 else None
        D = shifts(rng, 1, d)
        y = rng.standard_normal((1, nrhs, 2 ** int(m_r[r])))
        inst.append(dict(kind="dnet" if kinds[r] == 1 else "lattice", m=int(m_r[r]), lms=S,
                         shift=D, y=y))
    return dict(name="batched_256_mixed_d16", d=d, nrhs=nrhs, m_max=mmax, lattice_gen=g,
                net_gen=C, alpha=np.full(d, 2, np.int32),
                gamma=1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2, zeta=1.0,
                sigma2=1e-8, instances=inst)


def _w5() -> dict:
    rng = np.random.default_rng(5)
    m, d, R = 16, 64, 64
    C = net_generating_matrices(rng, d, m)
    S = lms_matrices(rng, R, d)
    D = shifts(rng, R, d)
    y = rng.standard_normal((R, 1, 2**m))
    return dict(name="net_m16_d64_r64_dsi2_grad", kind="dnet", order="natural", m=m, d=d,
                R=R, gen=C, lms=S, shift=D, alpha=np.full(d, 2, np.int32),
                gamma=1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2, zeta=1.0,
                sigma2=1e-3, y=y, nrhs=1)


def small_batch(seed: int, ms, kinds, d: int, nrhs: int, m_max: int) -> dict:
    """An instance table like workload 4 with chosen sizes and kinds (same
    draw order: generators, then per instance S (nets), shift, responses)."""
    rng = np.random.default_rng(seed)
    g = lattice_generating_vector(rng, d, m_max)
    C = net_generating_matrices(rng, d, m_max)
    inst = []
    for m, kind in zip(ms, kinds):
        S = lms_matrices(rng, 1, d) if kind == "dnet" else None
        D = shifts(rng, 1, d)
        y = rng.standard_normal((1, nrhs, 2 ** int(m)))
        inst.append(dict(kind=kind, m=int(m), lms=S, shift=D, y=y))
    return dict(name="batch", d=d, nrhs=nrhs, m_max=m_max, lattice_gen=g, net_gen=C,
                alpha=np.full(d, 2, np.int32),
                gamma=1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2, zeta=1.0,
                sigma2=1e-8, instances=inst)


def instance_workload(table: dict, i: int) -> dict:
    """Instance i of a table as a one-replication workload dict."""
    ins = table["instances"][i]
    lat = ins["kind"] == "lattice"
    return dict(kind=ins["kind"], order="natural", m=ins["m"], m_max=table["m_max"],
                d=table["d"], R=1, gen=table["lattice_gen"] if lat else table["net_gen"],
                lms=ins["lms"], shift=ins["shift"], alpha=table["alpha"], gamma=table["gamma"],
                zeta=table["zeta"], sigma2=table["sigma2"], y=ins["y"], nrhs=table["nrhs"])


def small_net(seed: int, m: int, d: int, R: int = 1, m_max: int | None = None,
              nrhs: int = 1) -> dict:
    """A random net instance of any size (LMS + digital shift)."""
    rng = np.random.default_rng(seed)
    mm = m if m_max is None else m_max
    C = net_generating_matrices(rng, d, mm)
    S = lms_matrices(rng, R, d)
    D = shifts(rng, R, d)
    y = rng.standard_normal((R, nrhs, 2**m))
    return dict(kind="dnet", m=m, m_max=mm, d=d, R=R, gen=C, lms=S, shift=D, y=y)


def small_lattice(seed: int, m: int, d: int, R: int = 1, m_max: int | None = None,
                  nrhs: int = 1) -> dict:
    """A random shifted-lattice instance of any size."""
    rng = np.random.default_rng(seed)
    mm = m if m_max is None else m_max
    g = lattice_generating_vector(rng, d, mm)
    D = shifts(rng, R, d)
    y = rng.standard_normal((R, nrhs, 2**m))
    return dict(kind="lattice", m=m, m_max=mm, d=d, R=R, gen=g, lms=None, shift=D, y=y)


def cubature_weights(seed: int, R: int, nw: int, n: int) -> np.ndarray:
    """Random cubature weights [R][nw][n] scattered around the equal weights
    1/n (relative spread 1/2); row 0 of every replication is exactly 1/n."""
    rng = np.random.default_rng(seed)
    w = (1.0 + 0.5 * rng.standard_normal((R, nw, n))) / n
    if nw:
        w[:, 0, :] = 1.0 / n
    return w


def corner_peak_coefficients(d: int) -> np.ndarray:
    """Coefficients of the corner-peak test integrand of the RQMC example:
    c_j proportional to 1/j^2, scaled to sum to 1/4."""
    ct = 1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2
    return 0.25 * ct / ct.sum()


# ---------------------------------------------------------------------------
# Point sets in prime bases (Halton, Faure) and nested uniform scrambling
# ---------------------------------------------------------------------------
B_TMAX = 53  # digits per coordinate in the scramble layouts (2^53 >= b^T)


def _primes(count: int) -> list:
    """The first `count` primes (to size the random digits of each base)."""
    out, c = [], 2
    while len(out) < count:
        if all(c % p for p in out if p * p <= c):
            out.append(c)
        c += 1
    return out


def bpoint_inputs(seed: int, kind: str, R: int, d: int, base: int = 0) -> dict:
    """Random scrambles for a Halton (base of dimension j = the j-th prime)
    or Faure (one prime `base`) point set, drawn for all 53 digit rows of
    every (replication, dimension) in the order LMS, permutations, shifts:

    * lms ``uint8[R][d][53][53]``: lower triangular, diagonal uniform in
      {1..b-1}, below it uniform in {0..b-1} (Matousek's scrambling, Sec. 4.3);
    * perm ``uint8[R][d][53][256]``: row t holds a uniform random permutation
      of {0..b-1} in its first b entries (digit permutations, Sec. 4.3);
    * shift ``uint8[R][d][53]``: uniform digits in {0..b-1}."""
    rng = np.random.default_rng(seed)
    bases = _primes(d) if kind == "halton" else [base] * d
    lms = np.zeros((R, d, B_TMAX, B_TMAX), np.uint8)
    perm = np.zeros((R, d, B_TMAX, 256), np.uint8)
    shift = np.zeros((R, d, B_TMAX), np.uint8)
    for r in range(R):
        for j in range(d):
            b = bases[j]
            low = rng.integers(0, b, size=(B_TMAX, B_TMAX))
            lms[r, j] = np.tril(low, -1) + np.diag(rng.integers(1, b, size=B_TMAX))
    for r in range(R):
        for j in range(d):
            b = bases[j]
            for t in range(B_TMAX):
                perm[r, j, t, :b] = rng.permutation(b)
    for r in range(R):
        for j in range(d):
            shift[r, j] = rng.integers(0, bases[j], size=B_TMAX)
    return dict(lms=lms, perm=perm, shift=shift)


def nus_seeds(seed: int, R: int, d: int) -> np.ndarray:
    """Seeds [R][d] of the nested uniform scrambling's counter-based flips."""
    return _u64(np.random.default_rng(seed), (R, d))
