"""CPU oracle for the fast kernel-method path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: its arithmetic is plain C in ``orc_*.c`` (built with gcc into
``liborc.so``) plus the exact-rational brute-force layer in ``brute.py``.

What it computes, and what pins each part (tests marked ``not gpu``):

=====================  =====================================================
lattice points         Sec. 4.2; natural == linear order element-wise via
                       R_m(i) and as sets (stated in Sec. 4.2); g = 1 gives
                       the van der Corput sequence
net points             Sec. 4.3; GF(2) brute force on unpacked digits;
                       stratification of the leading m digits; identity C
                       gives van der Corput; Gray order vs Table 1
interlacing            Sec. 4.3; the printed interlacing example (every
                       position's source entry); alpha = 1 is the identity;
                       the interlaced net's points are the digit-interlaced
                       points of the alpha d-dimensional net
SI factor              Sec. 5.2; truncated Fourier series with a tail bound;
                       special values pi^2/3, -pi^2/6, pi^4/45, ...
DSI factors a=2,3,4    Theorem 1; exact-rational Walsh series (eq. DSI_kernel)
                       organised as in Appendix B; s~_4(0) = 1/294 (App. B);
                       Walsh convention pinned by the Lemma of App. B
DSI factor a=1         PARITY UNPINNED (reading K_1 = 1 - 3 t_1); pinned only
                       by its own Walsh series
FWHT / FFTBR / IFFTBR  Figure 3; direct O(n^2) Hadamard and W^{k R(j)} matrices;
                       numpy FFT of the linear-order sequence; involution /
                       inverse
eig                    Sec. 5.4; closed-form Walsh / Fourier aliasing sums for
                       d = 1; circulant / RSBT structure of the dense Gram
solve, matvec, logdet  Sec. 5.4; dense Gram + Cholesky (numpy) at n <= 2^10
update_double          Sec. 5.4 / eq. (ft_next_parts); equals the fresh
                       transform of length 2n
MLL and gradient       standard GP objective in the eigenbasis of Sec. 5.4
                       (the paper prints none); dense GP likelihood and
                       trace-form gradient (numpy) at n <= 2^8; central
                       differences; adjoint dot-product identity; a factor
                       1 + gamma K that is exactly zero
kernel cubature        Sec. 3.2 (worst-case error, optimal
                       weights) and Bayesian cubature (Secs. 1.1, 1.3; no
                       formula printed: standard Gaussian conditioning); equal
                       weights in d = 1 against the aliased Fourier / Walsh
                       closed forms; each kernel factor has mean zero on
                       fine grids (kappa_i = zeta); stationarity of the
                       optimal weights; exact posterior mean on kernel
                       sections; eigenvalue forms equal the dense ones
Halton / Faure points  Secs. 4.3 (prime base) and 4.4; exact-rational radical
                       inverse; the (0, m, s)-net property of Faure (every
                       elementary interval of volume b^-m holds one point)
                       by brute force, kept by LMS; Faure's first dimension
                       is van der Corput; DS and DP undone by their
                       inverses give the unrandomized digits
NUS (base 2)           Sec. 4.3; digit t depends only on the digits before
                       it (points sharing a prefix share the scrambled
                       prefix), every level is a bijection, and the net's
                       stratification survives; the flips are balanced
RQMC estimate + CI     eq. (RQMC); Genz corner peak against its exact
                       integral (a one-dimensional Laplace-transform
                       quadrature, itself checked against inclusion-
                       exclusion) and the paper's printed estimate and
                       interval (Sec. 6 listing); Koksma-Hlawka bound in
                       d = 1; oscillatory rule on g = 1 in closed form;
                       the interval against scipy's t.interval
=====================  =====================================================
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_SRC = ["orc_points.c", "orc_kernels.c", "orc_algebra.c", "orc_mll.c", "orc_mll_ld.c",
        "orc_bpoints.c"]

LATTICE, DNET = 0, 1
NATURAL, LINEAR, GRAY = 0, 1, 2


def build(force: bool = True, path: str | None = None, flags=("-O2",)) -> str:
    """Compile the C oracle with gcc into oracle/liborc.so (or `path`).
    flags: optimisation flags; the CPU-baseline timing builds a copy with
    -O3 -march=native -fopenmp on the host that times it (the OpenMP
    pragmas only share out independent loops: results are bit for bit the
    same)."""
    out = path or _SO
    if force or not os.path.exists(out):
        cmd = ["gcc", *flags, "-std=gnu11", "-Wall", "-Wno-unknown-pragmas", "-fPIC", "-shared",
               "-o", out + ".tmp"]
        cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


_lib = None


def use_library(path: str | None):
    """Bind this module's functions to another build of the oracle (for the
    CPU-baseline timing); None returns to oracle/liborc.so."""
    global _lib
    _lib = None
    if path is not None:
        _lib = _load(path)


def lib():
    global _lib
    if _lib is None:
        newest_src = max(os.path.getmtime(os.path.join(_HERE, s))
                         for s in _SRC + ["orc.h", "orc_algebra.inc", "orc_kernels.inc"])
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < newest_src:
            build()
        _lib = _load(_SO)
    return _lib


def _load(path: str):
    """Load one build of the oracle and declare its signatures."""
    if True:
        L = C.CDLL(path)
        P = C.c_void_p
        i32, i64, f64 = C.c_int, C.c_int64, C.c_double
        sig = {
            "orc_lattice_points": [i32, i32, i32, i32, i64, i64, P, P, P],
            "orc_dnet_points": [i32, i32, i32, i32, i64, i64, P, P, P, P],
            "orc_lms": [i32, i32, P, P, P],
            "orc_kernel_column": [i32, i32, i32, i64, P, P, P, P, f64, P],
            "orc_fwht": [i64, P], "orc_fftbr": [i64, P], "orc_ifftbr": [i64, P],
            "orc_transform": [i32, i32, i32, i32, P, P],
            "orc_transform_ld": [i32, i32, i32, i32, P, P],
            "orc_eig": [i32, i32, i32, P, P, P], "orc_eig_ld": [i32, i32, i32, P, P],
            "orc_solve": [i32, i32, i32, i32, P, f64, P, P],
            "orc_solve_ld": [i32, i32, i32, i32, P, f64, P, P],
            "orc_matvec": [i32, i32, i32, i32, P, P, P],
            "orc_matvec_ld": [i32, i32, i32, i32, P, P, P],
            "orc_logdet": [i32, i32, P, f64, P], "orc_logdet_ld": [i32, i32, P, f64, P],
            "orc_update_double": [i32, i32, i32, P, P, P],
            "orc_eig_update_double": [i32, i32, i32, P, P, P],
            "orc_mll": [i32, i32, i32, P, f64, P, P, P, P],
            "orc_mll_adjoint": [i32, i32, i32, P, P],
            "orc_kernel_grad": [i32, i32, i32, i64, P, P, P, P, f64, P, P],
            "orc_mll_grad_ld": [i32, i32, i32, i32, P, P, P, P, f64, f64, P, P, P],
            "orc_bpoints": [i32, i32, i32, i32, i32, i64, i64, P, P, P, P],
            "orc_nus_points": [i32, i32, i32, i64, i64, P, P, P],
            "orc_bdigits": [i32], "orc_nth_prime": [i32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int if name not in ("orc_fwht", "orc_fftbr", "orc_ifftbr") else None
        L.orc_si_factor.argtypes = [i32, C.c_uint64]
        L.orc_si_factor.restype = f64
        L.orc_dsi_factor.argtypes = [i32, C.c_uint64]
        L.orc_dsi_factor.restype = f64
        L.orc_gray.argtypes = [C.c_uint64]
        L.orc_gray.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_mix64.restype = C.c_uint64
        L.orc_threads.argtypes = []
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        return L


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def kind_code(kind) -> int:
    return {"lattice": LATTICE, "dnet": DNET, LATTICE: LATTICE, DNET: DNET}[kind]


def order_code(order) -> int:
    return {"natural": NATURAL, "linear": LINEAR, "gray": GRAY,
            NATURAL: NATURAL, LINEAR: LINEAR, GRAY: GRAY}[order]


# ---------------------------------------------------------------------------
# Points
# ---------------------------------------------------------------------------

def lattice_points(g, shift, m: int, n_min: int, n_max: int, order="natural") -> np.ndarray:
    g = _c(g, np.uint64)
    shift = _c(shift, np.uint64)
    R = 1 if shift is None else shift.shape[0]
    d = g.shape[0]
    out = np.empty((R, n_max - n_min, d), dtype=np.uint64)
    _check(lib().orc_lattice_points(R, d, m, order_code(order), n_min, n_max, _p(g),
                                    _p(shift), _p(out)), "lattice_points")
    return out


def dnet_points(C_, S, shift, m_max: int, n_min: int, n_max: int, order="natural",
                R: int | None = None) -> np.ndarray:
    C_ = _c(C_, np.uint64)
    S = _c(S, np.uint64)
    shift = _c(shift, np.uint64)
    d = C_.shape[0]
    if R is None:
        R = S.shape[0] if S is not None else (shift.shape[0] if shift is not None else 1)
    out = np.empty((R, n_max - n_min, d), dtype=np.uint64)
    _check(lib().orc_dnet_points(R, d, m_max, order_code(order), n_min, n_max, _p(C_),
                                 _p(S), _p(shift), _p(out)), "dnet_points")
    return out


def lms(C_, S1) -> np.ndarray:
    """Scrambled generating matrices S_j C_j for one replication (S1: [d][64])."""
    C_ = _c(C_, np.uint64)
    S1 = _c(S1, np.uint64)
    out = np.empty_like(C_)
    _check(lib().orc_lms(C_.shape[0], C_.shape[1], _p(C_), _p(S1), _p(out)), "lms")
    return out


def interlace(cols, alpha: int) -> np.ndarray:
    """Digital interlacing (Sec. 4.3, higher-order nets).  cols =
    uint64[alpha d][m]: the columns of alpha d generating matrices (row t of
    column k at bit 63 - t).  Returns uint64[d][m]: row t of interlaced
    matrix j is row floor(t / alpha) of matrix alpha j + (t mod alpha)
    (0-based j), for the 64 rows a coordinate word holds.  Written on the
    unpacked digit matrices, entry by entry as the definition reads."""
    cols = np.ascontiguousarray(cols, dtype=np.uint64)
    ad, m = cols.shape
    if ad % alpha:
        raise ValueError("the number of matrices must be a multiple of alpha")
    d = ad // alpha
    shifts = (63 - np.arange(64)).astype(np.uint64)
    A = (cols[:, None, :] >> shifts[None, :, None]) & np.uint64(1)  # A[s][t][k]
    out = np.zeros((d, m), dtype=np.uint64)
    for j in range(d):
        for t in range(64):
            row = A[alpha * j + t % alpha, t // alpha, :]
            out[j] |= row << np.uint64(63 - t)
    return out


def interlace_columns(C_, S, alpha: int, R: int | None = None) -> np.ndarray:
    """Higher-order LMS (Sec. 4.3): scramble the alpha d source matrices of
    each replication (S[r], or none), then interlace: uint64[R][d][m]."""
    C_ = np.ascontiguousarray(C_, dtype=np.uint64)
    if R is None:
        R = 1 if S is None else S.shape[0]
    return np.stack([interlace(lms(C_, S[r]) if S is not None else C_, alpha)
                     for r in range(R)])


def higher_order_dnet_points(C_, S, shift, alpha: int, m_max: int, n_min: int, n_max: int,
                             order="natural") -> np.ndarray:
    """Points of a higher-order LMS + digitally shifted net: the d-dimensional
    net of every replication's interlaced scrambled matrices, shifted by its
    own shift[r] (d digits)."""
    R = S.shape[0] if S is not None else (shift.shape[0] if shift is not None else 1)
    cols = interlace_columns(C_, S, alpha, R)
    return np.stack([dnet_points(cols[r], None, None if shift is None else shift[r:r + 1],
                                 m_max, n_min, n_max, order, R=1)[0] for r in range(R)])


def gray(i: int) -> int:
    return int(lib().orc_gray(i))


def points(w: dict, n_min: int = 0, n_max: int | None = None, order=None) -> np.ndarray:
    """Points of a workload dict (see ``workloads``)."""
    m_max = w.get("m_max", w["m"])
    n_max = 2 ** w["m"] if n_max is None else n_max
    order = order or w.get("order", "natural")
    if w["kind"] == "lattice":
        return lattice_points(w["gen"], w["shift"], m_max, n_min, n_max, order)
    return dnet_points(w["gen"], w["lms"], w["shift"], m_max, n_min, n_max, order,
                       R=w["R"])


# ---------------------------------------------------------------------------
# Kernels
# ---------------------------------------------------------------------------

def si_factor(alpha: int, delta: int) -> float:
    return lib().orc_si_factor(alpha, int(delta))


def dsi_factor(alpha: int, delta: int) -> float:
    return lib().orc_dsi_factor(alpha, int(delta))


def kernel_column(kind, pts, x0, alpha, gamma, zeta: float) -> np.ndarray:
    pts = _c(pts, np.uint64)
    x0 = _c(x0, np.uint64)
    R, n, d = pts.shape
    alpha = _c(alpha, np.int32)
    gamma = _c(gamma, np.float64)
    out = np.empty((R, n), dtype=np.float64)
    _check(lib().orc_kernel_column(kind_code(kind), R, d, n, _p(pts), _p(x0), _p(alpha),
                                   _p(gamma), float(zeta), _p(out)), "kernel_column")
    return out


# ---------------------------------------------------------------------------
# Transforms and Gram algebra
# ---------------------------------------------------------------------------

def fwht(x) -> np.ndarray:
    x = np.array(x, dtype=np.float64, copy=True)
    lib().orc_fwht(x.shape[-1], _p(x))
    return x


def fftbr(x) -> np.ndarray:
    x = np.array(x, dtype=np.complex128, copy=True)
    lib().orc_fftbr(x.shape[-1], _p(x))
    return x


def ifftbr(x) -> np.ndarray:
    x = np.array(x, dtype=np.complex128, copy=True)
    lib().orc_ifftbr(x.shape[-1], _p(x))
    return x


def transform(kind, x, inverse: bool = False, precise: bool = False) -> np.ndarray:
    """Batched FFTBR/IFFTBR (lattice, complex) or FWHT (net, real) over the last axis."""
    k = kind_code(kind)
    dt = np.complex128 if k == LATTICE else np.float64
    x = _c(x, dt)
    n = x.shape[-1]
    m = n.bit_length() - 1
    B = x.size // n
    out = np.empty_like(x)
    fn = lib().orc_transform_ld if precise else lib().orc_transform
    _check(fn(k, -1 if inverse else 1, B, m, _p(x), _p(out)), "transform")
    return out


def eig(kind, k1, precise: bool = False):
    k1 = _c(k1, np.float64)
    R, n = k1.shape
    m = n.bit_length() - 1
    lam = np.empty_like(k1)
    if precise:
        _check(lib().orc_eig_ld(kind_code(kind), R, m, _p(k1), _p(lam)), "eig_ld")
        return lam
    mi = np.zeros(1)
    _check(lib().orc_eig(kind_code(kind), R, m, _p(k1), _p(lam), _p(mi)), "eig")
    return lam, float(mi[0])


def solve(kind, lam, sigma2: float, y, precise: bool = False) -> np.ndarray:
    lam = _c(lam, np.float64)
    y = _c(y, np.float64)
    R, nrhs, n = y.shape
    m = n.bit_length() - 1
    c = np.empty_like(y)
    fn = lib().orc_solve_ld if precise else lib().orc_solve
    _check(fn(kind_code(kind), R, nrhs, m, _p(lam), float(sigma2), _p(y), _p(c)), "solve")
    return c


def matvec(kind, lam, y, precise: bool = False) -> np.ndarray:
    lam = _c(lam, np.float64)
    y = _c(y, np.float64)
    R, nrhs, n = y.shape
    m = n.bit_length() - 1
    out = np.empty_like(y)
    fn = lib().orc_matvec_ld if precise else lib().orc_matvec
    _check(fn(kind_code(kind), R, nrhs, m, _p(lam), _p(y), _p(out)), "matvec")
    return out


def logdet(lam, sigma2: float, precise: bool = False) -> np.ndarray:
    lam = _c(lam, np.float64)
    R, n = lam.shape
    m = n.bit_length() - 1
    out = np.empty(R, dtype=np.float64)
    fn = lib().orc_logdet_ld if precise else lib().orc_logdet
    rc = fn(R, m, _p(lam), float(sigma2), _p(out))
    if rc not in (0, -4):
        _check(rc, "logdet")
    return out


def update_double(kind, yt_old, y_new) -> np.ndarray:
    k = kind_code(kind)
    y_new = _c(y_new, np.float64)
    B, n = y_new.shape
    m = n.bit_length() - 1
    yt_old = _c(yt_old, np.complex128 if k == LATTICE else np.float64)
    out = np.empty((B, 2 * n), dtype=yt_old.dtype)
    _check(lib().orc_update_double(k, B, m, _p(yt_old), _p(y_new), _p(out)), "update_double")
    return out


def eig_update_double(kind, lam_old, k1_new) -> np.ndarray:
    lam_old = _c(lam_old, np.float64)
    k1_new = _c(k1_new, np.float64)
    R, n = lam_old.shape
    m = n.bit_length() - 1
    out = np.empty((R, 2 * n), dtype=np.float64)
    _check(lib().orc_eig_update_double(kind_code(kind), R, m, _p(lam_old), _p(k1_new),
                                       _p(out)), "eig_update_double")
    return out


def fit_solve(w: dict, y=None, precise: bool = False) -> dict:
    """Whole path for one workload: points -> k1 -> lambda -> c, logdet."""
    pts = points(w)
    x0 = points(w, 0, 1)[:, 0, :]
    k1 = kernel_column(w["kind"], pts, x0, w["alpha"], w["gamma"], w["zeta"])
    lam, mi = eig(w["kind"], k1)
    y = w["y"] if y is None else y
    c = solve(w["kind"], lam, w["sigma2"], y)
    ld = logdet(lam, w["sigma2"])
    out = dict(pts=pts, k1=k1, lam=lam, max_imag=mi, c=c, logdet=ld)
    if precise:
        lam_ld = eig(w["kind"], k1, precise=True)
        out["lam_ld"] = lam_ld
        out["c_ld"] = solve(w["kind"], lam_ld, w["sigma2"], y, precise=True)
        out["logdet_ld"] = logdet(lam_ld, w["sigma2"], precise=True)
    return out


# ---------------------------------------------------------------------------
# GP marginal likelihood and gradient (one response per replication)
# ---------------------------------------------------------------------------

def mll(kind, lam, sigma2: float, y):
    """(L[R], g[R][n] = dL/dlambda, dL/dlog sigma2 [R]) for y: [R][n]."""
    lam = _c(lam, np.float64)
    y = _c(y, np.float64)
    R, n = lam.shape
    m = n.bit_length() - 1
    L = np.empty(R)
    g = np.empty_like(lam)
    ds = np.empty(R)
    _check(lib().orc_mll(kind_code(kind), R, m, _p(lam), float(sigma2), _p(y), _p(L), _p(g),
                         _p(ds)), "mll")
    return L, g, ds


def mll_adjoint(kind, g) -> np.ndarray:
    """dL/dk1 from dL/dlambda (adjoint of lambda = sqrt(n) FT(k1))."""
    g = _c(g, np.float64)
    R, n = g.shape
    a = np.empty_like(g)
    _check(lib().orc_mll_adjoint(kind_code(kind), R, n.bit_length() - 1, _p(g), _p(a)),
           "mll_adjoint")
    return a


def kernel_grad(kind, pts, x0, alpha, gamma, zeta: float, a) -> np.ndarray:
    """[R][d + 1]: sum_i a_i dk1_i/dlog gamma_j (j < d) and sum_i a_i k1_i (log zeta)."""
    pts = _c(pts, np.uint64)
    x0 = _c(x0, np.uint64)
    R, n, d = pts.shape
    a = _c(a, np.float64)
    out = np.empty((R, d + 1))
    _check(lib().orc_kernel_grad(kind_code(kind), R, d, n, _p(pts), _p(x0),
                                 _p(_c(alpha, np.int32)), _p(_c(gamma, np.float64)),
                                 float(zeta), _p(a), _p(out)), "kernel_grad")
    return out


def mll_grad(w: dict, gamma=None, zeta=None, sigma2=None, y=None) -> dict:
    """Whole gradient step for a workload: L[R] and grad[R][d + 2] in
    (log gamma_1..d, log zeta, log sigma2); replications share the parameters."""
    gamma = w["gamma"] if gamma is None else gamma
    zeta = w["zeta"] if zeta is None else zeta
    sigma2 = w["sigma2"] if sigma2 is None else sigma2
    y = w["y"][:, 0, :] if y is None else y
    pts = points(w)
    x0 = points(w, 0, 1)[:, 0, :]
    k1 = kernel_column(w["kind"], pts, x0, w["alpha"], gamma, zeta)
    lam, _ = eig(w["kind"], k1)
    L, g, ds = mll(w["kind"], lam, sigma2, y)
    a = mll_adjoint(w["kind"], g)
    kg = kernel_grad(w["kind"], pts, x0, w["alpha"], gamma, zeta, a)
    grad = np.concatenate([kg, ds[:, None]], axis=1)
    return dict(L=L, grad=grad, k1=k1, lam=lam, g=g, a=a)


def mll_grad_ld(w: dict, y=None) -> dict:
    """The same step as mll_grad with every intermediate in long double (an
    error reference only): L[R], grad[R][d + 2], rounded to double."""
    y = _c(w["y"][:, 0, :] if y is None else y, np.float64)
    pts = _c(points(w), np.uint64)
    x0 = _c(points(w, 0, 1)[:, 0, :], np.uint64)
    R, n, d = pts.shape
    L = np.empty(R)
    grad = np.empty((R, d + 2))
    _check(lib().orc_mll_grad_ld(kind_code(w["kind"]), R, d, n.bit_length() - 1, _p(pts), _p(x0),
                                 _p(_c(w["alpha"], np.int32)), _p(_c(w["gamma"], np.float64)),
                                 float(w["zeta"]), float(w["sigma2"]), _p(y), _p(L), _p(grad)),
           "mll_grad_ld")
    return dict(L=L, grad=grad)


# ---------------------------------------------------------------------------
# Kernel cubature: worst-case error, optimal weights, Bayesian cubature
# (Sec. 3.2; Bayesian cubature is named in Secs. 1.1 and 1.3)
# ---------------------------------------------------------------------------

def gram(kind, pts, alpha, gamma, zeta: float) -> np.ndarray:
    """Dense Gram matrices K[r][i][l] = K(x_ri, x_rl): column l is the kernel
    column anchored at point l (small n only)."""
    pts = _c(pts, np.uint64)
    R, n, d = pts.shape
    K = np.empty((R, n, n))
    for r in range(R):
        for l in range(n):
            K[r, :, l] = kernel_column(kind, pts[r:r + 1], pts[r:r + 1, l], alpha, gamma,
                                       zeta)[0]
    return K


def kernel_integrals(zeta: float, n: int):
    """kappa_i = int K(u, x_i) du (i < n) and int int K(u, v) du dv for the
    product kernel zeta prod_j (1 + gamma_j K_alpha(x_j (-) y_j)).  Each
    K_alpha has mean zero over [0, 1): the SI factor is a Bernoulli
    polynomial of degree 2 alpha (a Fourier series without constant term,
    Sec. 5.2) and the DSI factor a Walsh series without constant term
    (eq. DSI_kernel).  Hence every factor integrates to 1, whatever the
    other argument, and both integrals equal zeta."""
    return np.full(n, float(zeta)), float(zeta)


def wce2(K, kappa, I2: float, omega) -> np.ndarray:
    """Squared worst-case error of sum_i omega_i f(x_i) as an estimate of
    int f over the unit ball of the RKHS of K (Sec. 3.2):
    I2 - 2 sum_i omega_i kappa_i + sum_{i,l} omega_i omega_l K_il.
    K: [R][n][n]; omega: [R][nw][n]; returns [R][nw]."""
    K = np.asarray(K, np.float64)
    omega = np.asarray(omega, np.float64)
    kappa = np.asarray(kappa, np.float64)
    out = np.empty(omega.shape[:2])
    for r in range(omega.shape[0]):
        for q in range(omega.shape[1]):
            w = omega[r, q]
            out[r, q] = I2 - 2.0 * np.dot(w, kappa) + np.dot(w, K[r] @ w)
    return out


def wce2_fast(kind, lam, zeta: float, omega) -> np.ndarray:
    """The same squared worst-case error with K omega from the eigenvalue
    matvec (Sec. 5.4) and kappa_i = int int K = zeta (kernel_integrals)."""
    omega = _c(omega, np.float64)
    Kw = matvec(kind, lam, omega)
    return zeta - 2.0 * zeta * omega.sum(axis=-1) + (omega * Kw).sum(axis=-1)


def bayes_cubature(K, kappa, I2: float, y, sigma2: float) -> dict:
    """Posterior of I = int f for f ~ GP(0, s2 K) observed as y_i = f(x_i) +
    e_i, e_i ~ N(0, s2 sigma2), given the points (Bayesian cubature, named in
    Secs. 1.1 and 1.3; the paper prints no formula, so the Gaussian conditioning below is
    the standard one, with the scale s2 at its maximum-likelihood value):
      weights = (K + sigma2 I)^{-1} kappa       (the optimal cubature weights
                                                 omega* of Sec. kernel
                                                 computations when sigma2 = 0)
      mean    = kappa^T (K + sigma2 I)^{-1} y  = weights . y
      var     = I2 - kappa^T (K + sigma2 I)^{-1} kappa   (posterior variance / s2)
      s2      = y^T (K + sigma2 I)^{-1} y / n
      wce2    = squared worst-case error of the weights.
    K: [R][n][n]; y: [R][n].  Dense solves (numpy)."""
    K = np.asarray(K, np.float64)
    y = np.asarray(y, np.float64)
    kappa = np.asarray(kappa, np.float64)
    R, n = y.shape
    out = {k: np.empty(R) for k in ("mean", "var", "s2", "wce2")}
    out["weights"] = np.empty((R, n))
    for r in range(R):
        A = K[r] + sigma2 * np.eye(n)
        c = np.linalg.solve(A, y[r])
        wk = np.linalg.solve(A, kappa)
        out["weights"][r] = wk
        out["mean"][r] = np.dot(kappa, c)
        out["var"][r] = I2 - np.dot(kappa, wk)
        out["s2"][r] = np.dot(y[r], c) / n
    out["wce2"] = wce2(K, kappa, I2, out["weights"][:, None, :])[:, 0]
    return out


def bayes_cubature_fast(kind, lam, sigma2: float, zeta: float, y) -> dict:
    """bayes_cubature with the eigenvalue solve (Sec. 5.4) in place of the
    dense one and kappa = zeta (kernel_integrals).  lam: [R][n]; y: [R][n]."""
    lam = _c(lam, np.float64)
    y = _c(y, np.float64)
    R, n = y.shape
    kappa = np.full((R, 1, n), float(zeta))
    c = solve(kind, lam, sigma2, y[:, None, :])[:, 0]
    wk = solve(kind, lam, sigma2, kappa)[:, 0]
    return dict(weights=wk,
                mean=(kappa[:, 0] * c).sum(axis=-1),
                var=zeta - (kappa[:, 0] * wk).sum(axis=-1),
                s2=(y * c).sum(axis=-1) / n,
                wce2=wce2_fast(kind, lam, zeta, wk[:, None, :])[:, 0])


# ---------------------------------------------------------------------------
# RQMC estimate and Student-t interval (eq. RQMC), Genz test integrands
# ---------------------------------------------------------------------------

def unit_points(words) -> np.ndarray:
    """Coordinates of 64-bit fixed-point point words: u 2^-64 rounded to the
    nearest double."""
    return np.ldexp(np.asarray(words, dtype=np.uint64).astype(np.float64), -64)


def genz_corner_peak(x, c) -> np.ndarray:
    """Genz corner-peak integrand (1 + sum_j c_j x_j)^{-(d + 1)} over the last
    axis of x (the integrand of the paper's RQMC example, Sec. 6 listing)."""
    x = np.asarray(x, np.float64)
    d = x.shape[-1]
    return (1.0 + x @ np.asarray(c, np.float64)) ** (-(d + 1))


def genz_oscillatory(x, c, u: float) -> np.ndarray:
    """Genz oscillatory integrand cos(2 pi u + sum_j c_j x_j)."""
    x = np.asarray(x, np.float64)
    return np.cos(2.0 * np.pi * u + x @ np.asarray(c, np.float64))


def rqmc(y, tau: float = 0.01) -> dict:
    """eq. (RQMC): mu_r = mean over the n points of replication r, mu = mean
    of the mu_r, sigma^2 = sum_r (mu_r - mu)^2 / (R - 1), and the
    100(1 - tau)% interval mu +- t sigma / sqrt(R) with t the upper tau/2
    quantile of Student's t with R - 1 degrees of freedom (scipy).
    y: [R][n] integrand values."""
    from scipy import stats

    y = np.asarray(y, np.float64)
    R, n = y.shape
    mu_r = y.sum(axis=1) / n
    mu = mu_r.sum() / R
    sigma = math.sqrt(((mu_r - mu) ** 2).sum() / (R - 1)) if R > 1 else float("nan")
    t = float(stats.t.ppf(1.0 - tau / 2.0, R - 1)) if R > 1 else float("nan")
    return dict(mu_r=mu_r, mean=mu, std=sigma, t=t, half=t * sigma / math.sqrt(R))


# ---------------------------------------------------------------------------
# Point sets without FWHT structure (orc_bpoints.c)
# ---------------------------------------------------------------------------
BR_LMS, BR_DP, BR_DS = 1, 2, 4
BT_MAX = 53
_BKIND = {"halton": 2, "faure": 3}


def bdigits(b: int) -> int:
    """Digits kept in base b: the largest T with b^T <= 2^53."""
    return int(lib().orc_bdigits(int(b)))


def nth_prime(j: int) -> int:
    return int(lib().orc_nth_prime(int(j)))


def bpoints(kind: str, R: int, d: int, n_min: int, n_max: int, base: int = 0, flags: int = 0,
            lms=None, perm=None, shift=None) -> np.ndarray:
    """Coordinates [R][n][d] (FP64) of a Halton or Faure point set with the
    randomizations in `flags` (BR_LMS, then BR_DP, then BR_DS)."""
    cnt = n_max - n_min
    out = np.empty((R, cnt, d), np.float64)
    lms_ = None if lms is None else _c(lms, np.uint8)
    perm_ = None if perm is None else _c(perm, np.uint8)
    shift_ = None if shift is None else _c(shift, np.uint8)
    _check(lib().orc_bpoints(_BKIND[kind], R, d, int(base), int(flags), n_min, n_max,
                             _p(lms_), _p(perm_), _p(shift_), _p(out)), "bpoints")
    return out


def mix64(z: int) -> int:
    return int(lib().orc_mix64(C.c_uint64(int(z) & (2**64 - 1))))


def nus_points(C_, seed, m: int, n_min: int, n_max: int) -> np.ndarray:
    """Point words [R][n][d] of a base-2 net with generating columns C_ [d][m]
    under nested uniform scrambling with seeds [R][d]."""
    C_ = _c(C_, np.uint64)
    seed = _c(seed, np.uint64)
    R, d = seed.shape
    out = np.empty((R, n_max - n_min, d), np.uint64)
    _check(lib().orc_nus_points(R, d, m, n_min, n_max, _p(C_), _p(seed), _p(out)), "nus_points")
    return out
