"""Fast kernel methods on randomized low-discrepancy point sets, on MI355X.

Python binding of ``libldk.so`` (C ABI in ``include/ldk.h``).  The binding
only marshals arguments: every step runs in the library's HIP kernels, on
the current torch stream.  Torch tensors provide device memory; 64-bit
coordinate words are held in ``torch.int64`` tensors (bit patterns; view
them as uint64 on the host).

Raises ``LdkError`` if the library is missing or a call fails: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldk.so")

LATTICE, DNET_B2 = 0, 1
NATURAL, LINEAR, GRAY = 0, 1, 2
F64, F32 = 0, 1
GEN_PER_REPLICATION = 1
(OP_TRANSFORM, OP_EIG, OP_SOLVE, OP_MATVEC, OP_LOGDET, OP_UPDATE_DOUBLE, OP_EIG_UPDATE_DOUBLE,
 OP_MLL, OP_MLL_ADJOINT, OP_FIT, OP_WCE, OP_BAYES_CUBATURE) = range(12)
BC_FIELDS = ("mean", "var", "scale", "half", "weight", "wce2")
GENZ_CORNER_PEAK, GENZ_OSCILLATORY = 0, 1
RQMC_FIELDS = ("mean", "std", "half")

EXPORTS = [
    "ldk_init", "ldk_gen_points", "ldk_kernel_column", "ldk_transform", "ldk_eig", "ldk_solve",
    "ldk_matvec", "ldk_logdet", "ldk_update_double", "ldk_eig_update_double",
    "ldk_workspace_bytes", "ldk_strerror", "ldk_last_hip_error", "ldk_version",
    "ldk_mll", "ldk_mll_adjoint", "ldk_kernel_grad", "ldk_kernel_grad_workspace_bytes",
    "ldk_fwht_split16", "ldk_fit", "ldk_points_column", "ldk_interlace", "ldk_wce",
    "ldk_bayes_cubature", "ldk_rqmc", "ldk_rqmc_workspace_bytes", "ldk_solve_checked",
    "ldk_logdet_checked", "ldk_normal_quantile", "ldk_student_t_quantile", "ldk_solve_noalloc",
    "ldk_init_tuned", "ldk_plan_info", "ldk_plan_create", "ldk_plan_arena_bytes",
    "ldk_plan_instance_offset", "ldk_plan_bind", "ldk_batch_launch", "ldk_batch_capture",
    "ldk_plan_stats", "ldk_plan_destroy", "ldk_gen_bpoints", "ldk_bpoints_workspace_bytes",
    "ldk_rqmc_points", "ldk_rqmc_points_workspace_bytes",
]


class LdkError(RuntimeError):
    pass


class _Pointset(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.c_int32), ("R", C.c_int32), ("d", C.c_int32),
                ("m_max", C.c_int32), ("flags", C.c_int32), ("gen", C.c_void_p),
                ("lms", C.c_void_p), ("shift", C.c_void_p)]


class _BPointset(C.Structure):
    _fields_ = [("kind", C.c_int32), ("R", C.c_int32), ("d", C.c_int32), ("base", C.c_int32),
                ("flags", C.c_int32), ("m", C.c_int32), ("lms", C.c_void_p), ("perm", C.c_void_p),
                ("shift", C.c_void_p), ("gen", C.c_void_p), ("seed", C.c_void_p)]


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("alpha", C.c_void_p),
                ("gamma", C.c_void_p), ("zeta", C.c_double)]


_lib = None


def lib():
    """Load libldk.so (built by ``paper_2502_14256_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LdkError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f64 = C.c_void_p, C.c_int, C.c_int64, C.c_double
        sig = {
            "ldk_init": ([], i32),
            "ldk_gen_points": ([P, i64, i64, P, P], i32),
            "ldk_kernel_column": ([P, P, P, P, i64, i64, i32, P, P], i32),
            "ldk_points_column": ([P, P, i64, i64, P, i32, P, P], i32),
            "ldk_interlace": ([P, i32, P, P], i32),
            "ldk_wce": ([i32, i32, i32, i32, i32, P, f64, P, P, P, P], i32),
            "ldk_bayes_cubature": ([i32, i32, i32, i32, P, f64, f64, P, f64, P, P, P], i32),
            "ldk_rqmc": ([P, i64, i32, P, f64, f64, P, P, P, P], i32),
            "ldk_rqmc_workspace_bytes": ([P, i64], C.c_size_t),
            "ldk_transform": ([i32, i32, i32, i32, i32, P, P, P, P], i32),
            "ldk_eig": ([i32, i32, i32, i32, P, P, P, P], i32),
            "ldk_solve": ([i32, i32, i32, i32, i32, P, f64, P, P, P, P], i32),
            "ldk_matvec": ([i32, i32, i32, i32, i32, P, P, P, P, P], i32),
            "ldk_logdet": ([i32, i32, P, f64, P, P, P], i32),
            "ldk_update_double": ([i32, i32, i32, i32, P, P, P, P, P], i32),
            "ldk_eig_update_double": ([i32, i32, i32, i32, P, P, P, P, P], i32),
            "ldk_workspace_bytes": ([i32, i32, i64, i32, i32], C.c_size_t),
            "ldk_strerror": ([i32], C.c_char_p),
            "ldk_last_hip_error": ([], i32),
            "ldk_version": ([], C.c_char_p),
            "ldk_mll": ([i32, i32, i32, i32, P, f64, P, P, P, P, P, P], i32),
            "ldk_mll_adjoint": ([i32, i32, i32, P, P, P, P], i32),
            "ldk_kernel_grad": ([P, P, P, P, i64, i64, i32, P, P, P, P, P], i32),
            "ldk_kernel_grad_workspace_bytes": ([i32, i32, i64, i64, i32], C.c_size_t),
            "ldk_fwht_split16": ([i32, i32, P, P, P], i32),
            "ldk_fit": ([i32, i32, i32, i32, i32, P, f64, P, P, P, P, P, P], i32),
            "ldk_solve_checked": ([i32, i32, i32, i32, i32, P, f64, P, P, P, P], i32),
            "ldk_logdet_checked": ([i32, i32, P, f64, P, P, P], i32),
            "ldk_normal_quantile": ([f64], f64),
            "ldk_student_t_quantile": ([f64, i32, P], i32),
            "ldk_solve_noalloc": ([i32, i32, i32, i32, i32, P, f64, P, P, P], i32),
            "ldk_init_tuned": ([C.c_char_p], i32),
            "ldk_plan_info": ([i32, i32, i32, i64, P, P, P, P], i32),
            "ldk_gen_bpoints": ([P, i64, i64, P, P, P], i32),
            "ldk_bpoints_workspace_bytes": ([P], C.c_size_t),
            "ldk_rqmc_points": ([i32, i64, i32, P, i32, P, f64, f64, P, P, P, P], i32),
            "ldk_rqmc_points_workspace_bytes": ([i32, i64], C.c_size_t),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().ldk_strerror(rc).decode()
        raise LdkError(f"{what}: {msg} (status {rc}, hip error {lib().ldk_last_hip_error()})")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(dt: torch.dtype) -> int:
    if dt in (torch.float64, torch.complex128):
        return F64
    if dt in (torch.float32, torch.complex64):
        return F32
    raise LdkError(f"unsupported dtype {dt}")


def _real(dtype_code: int):
    return torch.float64 if dtype_code == F64 else torch.float32


def _cplx(dtype_code: int):
    return torch.complex128 if dtype_code == F64 else torch.complex64


def _need(t: torch.Tensor, name: str, device=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise LdkError(f"{name} must be a contiguous device tensor")
    if device is not None and t.device != torch.device(device):
        raise LdkError(f"{name} is on {t.device}, expected {device}")


def _need_out(t: torch.Tensor, name: str, dtype: torch.dtype, shape, device):
    """A caller-supplied output: contiguous, on `device`, of `dtype` and
    exactly numel(shape) elements (the kernels write every one of them)."""
    _need(t, name, device)
    if t.dtype != dtype:
        raise LdkError(f"{name} must be {dtype}, got {t.dtype}")
    want = 1
    for s_ in shape:
        want *= int(s_)
    if t.numel() != want:
        raise LdkError(f"{name} holds {t.numel()} elements, expected {want} ({tuple(shape)})")


def _need_ws(ws, nbytes: int, device):
    """A workspace of at least nbytes bytes on `device` (allocated when None)."""
    nbytes = int(nbytes)
    if ws is None:
        return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device) if nbytes else None
    _need(ws, "ws", device)
    if ws.numel() * ws.element_size() < nbytes:
        raise LdkError(f"workspace holds {ws.numel() * ws.element_size()} bytes, "
                       f"{nbytes} needed")
    return ws


def _kind(kind) -> int:
    return {"lattice": LATTICE, "dnet": DNET_B2, LATTICE: LATTICE, DNET_B2: DNET_B2}[kind]


def _order(order) -> int:
    return {"natural": NATURAL, "linear": LINEAR, "gray": GRAY,
            NATURAL: NATURAL, LINEAR: LINEAR, GRAY: GRAY}[order]


def _workspace(op: int, kind: int, rows: int, m: int, dt: int, device, ws=None):
    return _need_ws(ws, lib().ldk_workspace_bytes(op, kind, rows, m, dt), device)


def init(tuned: str | None = None):
    """Build the twiddle tables; with `tuned`, also load that tuned-plan
    table (see ldk_init_tuned)."""
    _check(lib().ldk_init(), "ldk_init")
    if tuned is not None:
        load_tuned(tuned)


def load_tuned(path: str | None):
    """Replace the tuned-plan table with the file at `path` (None clears it)."""
    _check(lib().ldk_init_tuned(None if path is None else os.fsencode(path)), "ldk_init_tuned")


def plan_info(kind, dtype, m: int, rows: int) -> dict:
    """The plan a transform call would use: log_tile, radix, passes and
    engine (0 FP32/FP64 butterflies, 1 split-FP16 matrix cores)."""
    lt, rx, ps, en = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    dt = dtype if isinstance(dtype, int) else _dtype_code(dtype)
    _check(lib().ldk_plan_info(_kind(kind), dt, m, rows, C.byref(lt), C.byref(rx), C.byref(ps),
                               C.byref(en)), "ldk_plan_info")
    return {"log_tile": lt.value, "radix": rx.value, "passes": ps.value, "engine": en.value}


@dataclass
class PointSet:
    """A randomized point set (Sec. 4.2 lattice / Sec. 4.3 base-2 net).

    gen: int64 device tensor, lattice g[d] or net columns C[d][m_max]
    (C[R][d][m_max] with per_replication, e.g. from ``interlace``);
    lms: net scrambles S[R][d][64] or None; shift: [R][d] or None."""

    kind: str
    R: int
    d: int
    m_max: int
    gen: torch.Tensor
    lms: torch.Tensor | None = None
    shift: torch.Tensor | None = None
    order: str = "natural"
    per_replication: bool = False

    def _c(self) -> _Pointset:
        for name in ("gen", "lms", "shift"):
            t = getattr(self, name)
            if t is not None:
                _need(t, name)
        return _Pointset(_kind(self.kind), _order(self.order), self.R, self.d, self.m_max,
                         GEN_PER_REPLICATION if self.per_replication else 0,
                         _ptr(self.gen), _ptr(self.lms), _ptr(self.shift))


@dataclass
class Kernel:
    """Product-weight SI (lattice) or DSI (net) kernel.

    alpha: per-dimension orders (host sequence of ints; kept on the host);
    gamma: float64[d] device tensor of product weights; zeta > 0."""

    kind: str
    alpha: object
    gamma: torch.Tensor
    zeta: float = 1.0

    def __post_init__(self):
        import numpy as np

        a = self.alpha.cpu().numpy() if isinstance(self.alpha, torch.Tensor) else self.alpha
        self._alpha_host = np.ascontiguousarray(np.asarray(a, dtype=np.int32).ravel())

    def _c(self) -> _Kernel:
        _need(self.gamma, "gamma")
        return _Kernel(_kind(self.kind), int(self._alpha_host.size),
                       C.c_void_p(self._alpha_host.ctypes.data), _ptr(self.gamma),
                       float(self.zeta))


def _dev_of(ps: PointSet):
    return ps.gen.device


def _ps_checked(ps: PointSet):
    """The C struct of ps, its arrays checked for device and size."""
    dev = _dev_of(ps)
    per = ps.per_replication
    _need(ps.gen, "gen", dev)
    if ps.kind in ("lattice", LATTICE):
        want = ps.d
    else:
        want = ps.d * ps.m_max * (ps.R if per else 1)
    if ps.gen.numel() < want:
        raise LdkError(f"gen holds {ps.gen.numel()} words, {want} needed")
    if ps.lms is not None:
        _need(ps.lms, "lms", dev)
        if ps.lms.numel() < ps.R * ps.d * 64:
            raise LdkError("lms must hold S[R][d][64]")
    if ps.shift is not None:
        _need(ps.shift, "shift", dev)
        if ps.shift.numel() < ps.R * ps.d:
            raise LdkError("shift must hold [R][d] words")
    return ps._c()


def _k_checked(k: Kernel, d: int, dev):
    _need(k.gamma, "gamma", dev)
    if k.gamma.dtype != torch.float64 or k.gamma.numel() != d or k._alpha_host.size != d:
        raise LdkError("kernel gamma must be float64[d] and alpha hold d orders")
    return k._c()


def gen_points(ps: PointSet, n_min: int, n_max: int, out: torch.Tensor | None = None):
    dev = _dev_of(ps)
    shape = (ps.R, n_max - n_min, ps.d)
    if out is None:
        out = torch.empty(shape, dtype=torch.int64, device=dev)
    _need_out(out, "out", torch.int64, shape, dev)
    _check(lib().ldk_gen_points(C.byref(_ps_checked(ps)), n_min, n_max, _ptr(out), _stream()),
           "ldk_gen_points")
    return out


def kernel_column(k: Kernel, ps: PointSet, n_min: int, n_max: int, pts=None, x0=None,
                  dtype=torch.float64, out=None):
    dt = _dtype_code(dtype)
    dev = _dev_of(ps)
    shape = (ps.R, n_max - n_min)
    if out is None:
        out = torch.empty(shape, dtype=_real(dt), device=dev)
    _need_out(out, "out", _real(dt), shape, dev)
    if pts is not None:
        _need_out(pts, "pts", torch.int64, (ps.R, n_max - n_min, ps.d), dev)
    if x0 is not None:
        _need_out(x0, "x0", torch.int64, (ps.R, ps.d), dev)
    _check(lib().ldk_kernel_column(C.byref(_k_checked(k, ps.d, dev)), C.byref(_ps_checked(ps)),
                                   _ptr(pts), _ptr(x0), n_min, n_max, dt, _ptr(out), _stream()),
           "ldk_kernel_column")
    return out


def interlace(src: PointSet, alpha: int, shift: torch.Tensor | None = None, order=None,
              out: torch.Tensor | None = None) -> PointSet:
    """Higher-order net by digital interlacing (higher-order LMS when src has
    scrambles): src is a net of alpha d dimensions; returns the
    d-dimensional net whose per-replication generating columns are the
    interlaced scrambled ones (written to ``out``, int64 [R][d][m_max]),
    digitally shifted by ``shift`` ([R][d]) in ``order`` (src's by default)."""
    if src.d % alpha:
        raise LdkError("src.d must be a multiple of alpha")
    d = src.d // alpha
    dev = _dev_of(src)
    shape = (src.R, d, src.m_max)
    if out is None:
        out = torch.empty(shape, dtype=torch.int64, device=dev)
    _need_out(out, "out", torch.int64, shape, dev)
    _check(lib().ldk_interlace(C.byref(_ps_checked(src)), alpha, _ptr(out), _stream()),
           "ldk_interlace")
    return PointSet("dnet", src.R, d, src.m_max, out, None, shift, order or src.order,
                    per_replication=True)


def points_column(k: Kernel, ps: PointSet, n_min: int, n_max: int, dtype=torch.float64,
                  pts: torch.Tensor | None = None, k1: torch.Tensor | None = None):
    """(points, first column): gen_points and kernel_column (points
    regenerated) in one call, bit for bit the same outputs."""
    dt = _dtype_code(dtype)
    dev = _dev_of(ps)
    if pts is None:
        pts = torch.empty((ps.R, n_max - n_min, ps.d), dtype=torch.int64, device=dev)
    if k1 is None:
        k1 = torch.empty((ps.R, n_max - n_min), dtype=_real(dt), device=dev)
    _need_out(pts, "pts", torch.int64, (ps.R, n_max - n_min, ps.d), dev)
    _need_out(k1, "k1", _real(dt), (ps.R, n_max - n_min), dev)
    _check(lib().ldk_points_column(C.byref(_k_checked(k, ps.d, dev)), C.byref(_ps_checked(ps)),
                                   n_min, n_max, _ptr(pts), dt, _ptr(k1), _stream()),
           "ldk_points_column")
    return pts, k1


def _m_of(n: int) -> int:
    m = n.bit_length() - 1
    if n < 1 or n != 1 << m:
        raise LdkError(f"length {n} is not a power of two")
    return m


def transform(kind, x: torch.Tensor, inverse: bool = False, out=None):
    """FFTBR / IFFTBR (lattice, complex rows) or FWHT (net, real rows) over the last axis."""
    kd = _kind(kind)
    _need(x, "x")
    dt = _dtype_code(x.dtype)
    if (kd == LATTICE) != x.is_complex():
        raise LdkError("lattice transforms take complex rows, net transforms real rows")
    n = x.shape[-1]
    m = _m_of(n)
    B = x.numel() // n
    out = torch.empty_like(x) if out is None else out
    _need_out(out, "out", x.dtype, x.shape, x.device)
    ws = _workspace(OP_TRANSFORM, kd, B, m, dt, x.device)
    _check(lib().ldk_transform(kd, -1 if inverse else 1, B, m, dt, _ptr(x), _ptr(out), _ptr(ws),
                               _stream()), "ldk_transform")
    return out


def _need_f64(t: torch.Tensor, name: str, shape=None, device=None):
    _need(t, name, device)
    if t.dtype != torch.float64:
        raise LdkError(f"{name} must be float64 (eigenvalues are always FP64)")
    if shape is not None:
        _need_out(t, name, torch.float64, shape, t.device)


def eig(kind, k1: torch.Tensor, out=None, ws=None):
    """lambda = sqrt(n) FT(k1) in FP64 (k1 may be float32 or float64)."""
    kd = _kind(kind)
    _need(k1, "k1")
    dt = _dtype_code(k1.dtype)
    R, n = k1.shape
    m = _m_of(n)
    dev = k1.device
    out = torch.empty((R, n), dtype=torch.float64, device=dev) if out is None else out
    _need_out(out, "out", torch.float64, (R, n), dev)
    ws = _workspace(OP_EIG, kd, R, m, dt, dev, ws)
    _check(lib().ldk_eig(kd, R, m, dt, _ptr(k1), _ptr(out), _ptr(ws), _stream()), "ldk_eig")
    return out


def _apply_args(kind, lam, y, out, ws, op):
    kd = _kind(kind)
    _need(y, "y")
    dev = y.device
    dt = _dtype_code(y.dtype)
    if y.is_complex() or y.dim() != 3:
        raise LdkError("y must be a real [R][nrhs][n] tensor")
    R, nrhs, n = y.shape
    m = _m_of(n)
    _need_f64(lam, "lam", (R, n), dev)
    out = torch.empty_like(y) if out is None else out
    _need_out(out, "out", y.dtype, y.shape, dev)
    ws = _workspace(op, kd, R * nrhs, m, dt, dev, ws)
    return kd, dt, R, nrhs, m, out, ws


def solve(kind, lam: torch.Tensor, sigma2: float, y: torch.Tensor, out=None, ws=None,
          checked: bool = False):
    """c = (K + sigma2 I)^-1 y for y [R][nrhs][n] (ldk_solve).  With
    checked=True the call (ldk_solve_checked) also verifies on the device
    that every lambda_k + sigma2 > 0 and raises LdkError (status ENOTSPD)
    otherwise; it synchronises the stream."""
    kd, dt, R, nrhs, m, out, ws = _apply_args(kind, lam, y, out, ws, OP_SOLVE)
    fn = lib().ldk_solve_checked if checked else lib().ldk_solve
    _check(fn(kd, R, nrhs, m, dt, _ptr(lam), float(sigma2), _ptr(y), _ptr(out), _ptr(ws),
              _stream()), "ldk_solve_checked" if checked else "ldk_solve")
    return out


NOALLOC_SCRATCH_BYTES = 16 << 20  # LDK_NOALLOC_SCRATCH_BYTES


def solve_noalloc(kind, lam: torch.Tensor, sigma2: float, y: torch.Tensor, out: torch.Tensor):
    """ldk_solve_noalloc: the solve with its intermediates in the library's
    fixed per-GPU scratch (no workspace, no allocation in the library; the
    caller passes the output).  Raises LdkError (status -5) when the input
    needs more than NOALLOC_SCRATCH_BYTES of intermediates.  Calls that
    overlap on one GPU race."""
    kd = _kind(kind)
    _need(y, "y")
    dev = y.device
    if y.is_complex() or y.dim() != 3:
        raise LdkError("y must be a real [R][nrhs][n] tensor")
    R, nrhs, n = y.shape
    m = _m_of(n)
    _need_f64(lam, "lam", (R, n), dev)
    _need_out(out, "out", y.dtype, y.shape, dev)
    _check(lib().ldk_solve_noalloc(kd, R, nrhs, m, _dtype_code(y.dtype), _ptr(lam), float(sigma2),
                                   _ptr(y), _ptr(out), _stream()), "ldk_solve_noalloc")
    return out


def matvec(kind, lam: torch.Tensor, y: torch.Tensor, out=None, ws=None):
    kd, dt, R, nrhs, m, out, ws = _apply_args(kind, lam, y, out, ws, OP_MATVEC)
    _check(lib().ldk_matvec(kd, R, nrhs, m, dt, _ptr(lam), _ptr(y), _ptr(out), _ptr(ws),
                            _stream()), "ldk_matvec")
    return out


def logdet(lam: torch.Tensor, sigma2: float, out=None, ws=None, checked: bool = False):
    """log det(K + sigma2 I) per replication (ldk_logdet; ldk_logdet_checked
    with checked=True raises LdkError with status ENOTSPD instead of
    returning NaN, and synchronises the stream)."""
    _need_f64(lam, "lam")
    R, n = lam.shape
    m = _m_of(n)
    dev = lam.device
    out = torch.empty(R, dtype=torch.float64, device=dev) if out is None else out
    _need_out(out, "out", torch.float64, (R,), dev)
    ws = _workspace(OP_LOGDET, DNET_B2, R, m, F64, dev, ws)
    fn = lib().ldk_logdet_checked if checked else lib().ldk_logdet
    _check(fn(R, m, _ptr(lam), float(sigma2), _ptr(out), _ptr(ws), _stream()),
           "ldk_logdet_checked" if checked else "ldk_logdet")
    return out


def fit(kind, k1: torch.Tensor, sigma2: float, y: torch.Tensor, lam=None, c=None,
        logdet: bool | torch.Tensor = True, ws=None):
    """Eigenvalues, solves and log-det in one call: (lam, c, logdet or None).
    y: [R][nrhs][n] of k1's dtype."""
    kd = _kind(kind)
    _need(k1, "k1")
    dev = k1.device
    _need(y, "y", dev)
    dt = _dtype_code(k1.dtype)
    if y.dtype != k1.dtype:
        raise LdkError("k1 and y must share a dtype")
    R, n = k1.shape
    if y.dim() != 3 or y.shape[0] != R or y.shape[2] != n:
        raise LdkError("y must be [R][nrhs][n]")
    nrhs = y.shape[1]
    m = _m_of(n)
    lam = torch.empty((R, n), dtype=torch.float64, device=dev) if lam is None else lam
    _need_out(lam, "lam", torch.float64, (R, n), dev)
    c = torch.empty_like(y) if c is None else c
    _need_out(c, "c", y.dtype, y.shape, dev)
    ld = None
    if logdet is True:
        ld = torch.empty(R, dtype=torch.float64, device=dev)
    elif isinstance(logdet, torch.Tensor):
        ld = logdet
        _need_out(ld, "logdet", torch.float64, (R,), dev)
    ws = _workspace(OP_FIT, kd, R * (nrhs + 1), m, dt, dev, ws)
    _check(lib().ldk_fit(kd, R, nrhs, m, dt, _ptr(k1), float(sigma2), _ptr(y), _ptr(lam), _ptr(c),
                         _ptr(ld), _ptr(ws), _stream()), "ldk_fit")
    return lam, c, ld


def update_double(kind, yt_old: torch.Tensor, y_new: torch.Tensor, out=None):
    kd = _kind(kind)
    _need(y_new, "y_new")
    dev = y_new.device
    _need(yt_old, "yt_old", dev)
    dt = _dtype_code(y_new.dtype)
    B, n = y_new.shape
    m = _m_of(n)
    want = _cplx(dt) if kd == LATTICE else _real(dt)
    _need_out(yt_old, "yt_old", want, (B, n), dev)
    if out is None:
        out = torch.empty((B, 2 * n), dtype=want, device=dev)
    _need_out(out, "out", want, (B, 2 * n), dev)
    ws = _workspace(OP_UPDATE_DOUBLE, kd, B, m, dt, dev)
    _check(lib().ldk_update_double(kd, B, m, dt, _ptr(yt_old), _ptr(y_new), _ptr(out), _ptr(ws),
                                   _stream()), "ldk_update_double")
    return out


def eig_update_double(kind, lam_old: torch.Tensor, k1_new: torch.Tensor, out=None):
    kd = _kind(kind)
    _need_f64(lam_old, "lam_old")
    dev = lam_old.device
    _need(k1_new, "k1_new", dev)
    dt = _dtype_code(k1_new.dtype)
    R, n = lam_old.shape
    if tuple(k1_new.shape) != (R, n):
        raise LdkError("k1_new must be [R][n] like lam_old")
    m = _m_of(n)
    if out is None:
        out = torch.empty((R, 2 * n), dtype=torch.float64, device=dev)
    _need_out(out, "out", torch.float64, (R, 2 * n), dev)
    ws = _workspace(OP_EIG_UPDATE_DOUBLE, kd, R, m, dt, dev)
    _check(lib().ldk_eig_update_double(kd, R, m, dt, _ptr(lam_old), _ptr(k1_new), _ptr(out),
                                       _ptr(ws), _stream()), "ldk_eig_update_double")
    return out


# ---------------------------------------------------------------------------
# GP marginal likelihood and its gradient (one response per replication)
# ---------------------------------------------------------------------------

def mll(kind, lam: torch.Tensor, sigma2: float, y: torch.Tensor, out_g=None, ws=None):
    """(L[R], g[R][n] = dL/dlambda, dL/dlog sigma2 [R]) for y of shape [R][n]."""
    kd = _kind(kind)
    _need(y, "y")
    dev = y.device
    dt = _dtype_code(y.dtype)
    R, n = y.shape
    _need_f64(lam, "lam", (R, n), dev)
    m = _m_of(n)
    L = torch.empty(R, dtype=torch.float64, device=dev)
    ds = torch.empty(R, dtype=torch.float64, device=dev)
    g = torch.empty((R, n), dtype=torch.float64, device=dev) if out_g is None else out_g
    _need_out(g, "g", torch.float64, (R, n), dev)
    ws = _workspace(OP_MLL, kd, R, m, dt, dev, ws)
    _check(lib().ldk_mll(kd, R, m, dt, _ptr(lam), float(sigma2), _ptr(y), _ptr(L), _ptr(g),
                         _ptr(ds), _ptr(ws), _stream()), "ldk_mll")
    return L, g, ds


def wce(kind, lam: torch.Tensor, w: torch.Tensor, zeta: float, out=None, ws=None):
    """Squared worst-case errors [R][nw] of the cubature weights w [R][nw][n]
    for the product kernel with eigenvalues lam [R][n] (ldk_wce)."""
    kd = _kind(kind)
    _need(w, "w")
    dev = w.device
    dt = _dtype_code(w.dtype)
    R, nw, n = w.shape
    _need_f64(lam, "lam", (R, n), dev)
    m = _m_of(n)
    out = torch.empty((R, nw), dtype=torch.float64, device=dev) if out is None else out
    _need_out(out, "out", torch.float64, (R, nw), dev)
    ws = _workspace(OP_WCE, kd, R * nw, m, dt, dev, ws)
    _check(lib().ldk_wce(kd, R, nw, m, dt, _ptr(lam), float(zeta), _ptr(w), _ptr(out), _ptr(ws),
                         _stream()), "ldk_wce")
    return out


def normal_quantile(p: float) -> float:
    """Quantile of the standard normal distribution (ldk_normal_quantile:
    Abramowitz-Stegun 26.2.23 start, Halley steps on Phi through erfc)."""
    if not 0.0 < p < 1.0:
        raise LdkError("p must lie in (0, 1)")
    return float(lib().ldk_normal_quantile(float(p)))


def student_t_quantile(p: float, dof: int) -> float:
    """Quantile of Student's t distribution with dof degrees of freedom
    (ldk_student_t_quantile: Cornish-Fisher start, Newton steps on the
    upper tail through the regularised incomplete beta function)."""
    if not 0.0 < p < 1.0 or dof < 1:
        raise LdkError("p must lie in (0, 1) and dof >= 1")
    q = C.c_double(0.0)
    _check(lib().ldk_student_t_quantile(float(p), int(dof), C.byref(q)), "ldk_student_t_quantile")
    return q.value


def bayes_cubature(kind, lam: torch.Tensor, sigma2: float, zeta: float, y: torch.Tensor,
                   level: float = 0.99, out=None, ws=None):
    """Bayesian-cubature posterior of the integral per replication (ldk_bayes_cubature):
    a double tensor [R][6] whose columns are named by BC_FIELDS; the credible
    interval is mean +- half at the given level."""
    kd = _kind(kind)
    _need(y, "y")
    dev = y.device
    dt = _dtype_code(y.dtype)
    R, n = y.shape
    _need_f64(lam, "lam", (R, n), dev)
    if not 0.0 < level < 1.0:
        raise LdkError("level must lie in (0, 1)")
    m = _m_of(n)
    z = normal_quantile(0.5 + 0.5 * level)
    out = torch.empty((R, len(BC_FIELDS)), dtype=torch.float64, device=dev) \
        if out is None else out
    _need_out(out, "out", torch.float64, (R, len(BC_FIELDS)), dev)
    ws = _workspace(OP_BAYES_CUBATURE, kd, R, m, dt, dev, ws)
    _check(lib().ldk_bayes_cubature(kd, R, m, dt, _ptr(lam), float(sigma2), float(zeta), _ptr(y),
                                    float(z), _ptr(out), _ptr(ws), _stream()),
           "ldk_bayes_cubature")
    return out


def rqmc(ps: PointSet, n: int, integrand, coef: torch.Tensor, u: float = 0.0, tau: float = 0.01,
         mu_r=None, stats=None, ws=None):
    """RQMC estimate over the R randomizations of ps (ldk_rqmc): (mu_r [R],
    stats [3] = mean, std, half width of the 100(1 - tau)% Student-t
    interval).  integrand: "corner_peak" or "oscillatory" (or GENZ_*)."""
    f = {"corner_peak": GENZ_CORNER_PEAK, "oscillatory": GENZ_OSCILLATORY,
         GENZ_CORNER_PEAK: GENZ_CORNER_PEAK, GENZ_OSCILLATORY: GENZ_OSCILLATORY}[integrand]
    dev = _dev_of(ps)
    _need_f64(coef, "coef", (ps.d,), dev)
    if not 0.0 < tau < 1.0:
        raise LdkError("tau must lie in (0, 1)")
    t = student_t_quantile(1.0 - tau / 2.0, ps.R - 1) if ps.R > 1 else 0.0
    mu_r = torch.empty(ps.R, dtype=torch.float64, device=dev) if mu_r is None else mu_r
    stats = torch.empty(len(RQMC_FIELDS), dtype=torch.float64, device=dev) if stats is None \
        else stats
    _need_out(mu_r, "mu_r", torch.float64, (ps.R,), dev)
    _need_out(stats, "stats", torch.float64, (len(RQMC_FIELDS),), dev)
    cps = _ps_checked(ps)
    ws = _need_ws(ws, lib().ldk_rqmc_workspace_bytes(C.byref(cps), int(n)), dev)
    _check(lib().ldk_rqmc(C.byref(cps), int(n), f, _ptr(coef), float(u), t, _ptr(mu_r),
                          _ptr(stats), _ptr(ws), _stream()), "ldk_rqmc")
    return mu_r, stats


HALTON, FAURE, DNET_NUS = 2, 3, 4
BR_LMS, BR_DP, BR_DS = 1, 2, 4
BDIGITS_MAX = 53


@dataclass
class BPointSet:
    """A point set without fast-transform structure (ldk_gen_bpoints):
    kind "halton" (the j-th prime per dimension), "faure" (one prime base)
    or "nus" (nested uniform scrambling of a base-2 net with generating
    columns gen [d][m] and seeds [R][d]).  flags: OR of BR_LMS, BR_DP, BR_DS
    (Halton / Faure) with the uint8 scrambles lms [R][d][53][53], perm
    [R][d][53][256] and shift [R][d][53] on the device."""

    kind: str
    R: int
    d: int
    base: int = 0
    flags: int = 0
    lms: torch.Tensor | None = None
    perm: torch.Tensor | None = None
    shift: torch.Tensor | None = None
    gen: torch.Tensor | None = None
    seed: torch.Tensor | None = None
    m: int = 0

    def _c(self) -> _BPointset:
        kd = {"halton": HALTON, "faure": FAURE, "nus": DNET_NUS}[self.kind]
        R, d = self.R, self.d
        shapes = {"lms": ((R, d, BDIGITS_MAX, BDIGITS_MAX), torch.uint8),
                  "perm": ((R, d, BDIGITS_MAX, 256), torch.uint8),
                  "shift": ((R, d, BDIGITS_MAX), torch.uint8),
                  "gen": ((d, self.m), torch.int64), "seed": ((R, d), torch.int64)}
        for name, (shape, dt) in shapes.items():
            t = getattr(self, name)
            if t is not None:
                _need(t, name)
                if t.dtype != dt or tuple(t.shape) != shape:
                    raise LdkError(f"{name} must be {dt} of shape {shape}")
        return _BPointset(kd, R, d, int(self.base), int(self.flags), int(self.m), _ptr(self.lms),
                          _ptr(self.perm), _ptr(self.shift), _ptr(self.gen), _ptr(self.seed))


def gen_bpoints(ps: BPointSet, n_min: int, n_max: int, out=None, ws=None, device="cuda"):
    """Coordinates [R][n_max - n_min][d] (FP64) of a BPointSet (ldk_gen_bpoints)."""
    cps = ps._c()
    shape = (ps.R, n_max - n_min, ps.d)
    out = torch.empty(shape, dtype=torch.float64, device=device) if out is None else out
    _need_out(out, "out", torch.float64, shape, out.device)
    ws = _need_ws(ws, lib().ldk_bpoints_workspace_bytes(C.byref(cps)), out.device)
    _check(lib().ldk_gen_bpoints(C.byref(cps), int(n_min), int(n_max), _ptr(out), _ptr(ws),
                                 _stream()), "ldk_gen_bpoints")
    return out


def rqmc_points(x: torch.Tensor, integrand, coef: torch.Tensor, u: float = 0.0, tau: float = 0.01,
                mu_r=None, stats=None, ws=None):
    """RQMC estimate over given coordinates x [R][n][d] (ldk_rqmc_points):
    (mu_r [R], stats [3]) as rqmc."""
    f = {"corner_peak": GENZ_CORNER_PEAK, "oscillatory": GENZ_OSCILLATORY,
         GENZ_CORNER_PEAK: GENZ_CORNER_PEAK, GENZ_OSCILLATORY: GENZ_OSCILLATORY}[integrand]
    _need_f64(x, "x")
    R, n, d = x.shape
    dev = x.device
    _need_f64(coef, "coef", (d,), dev)
    if not 0.0 < tau < 1.0:
        raise LdkError("tau must lie in (0, 1)")
    t = student_t_quantile(1.0 - tau / 2.0, R - 1) if R > 1 else 0.0
    mu_r = torch.empty(R, dtype=torch.float64, device=dev) if mu_r is None else mu_r
    stats = torch.empty(len(RQMC_FIELDS), dtype=torch.float64, device=dev) if stats is None \
        else stats
    _need_out(mu_r, "mu_r", torch.float64, (R,), dev)
    _need_out(stats, "stats", torch.float64, (len(RQMC_FIELDS),), dev)
    ws = _need_ws(ws, lib().ldk_rqmc_points_workspace_bytes(R, n), dev)
    _check(lib().ldk_rqmc_points(R, n, d, _ptr(x), f, _ptr(coef), float(u), t, _ptr(mu_r),
                                 _ptr(stats), _ptr(ws), _stream()), "ldk_rqmc_points")
    return mu_r, stats


def mll_adjoint(kind, g: torch.Tensor, out=None, ws=None):
    """dL/dk1 from dL/dlambda (adjoint of lambda = sqrt(n) FT(k1)), FP64."""
    kd = _kind(kind)
    _need_f64(g, "g")
    R, n = g.shape
    m = _m_of(n)
    dev = g.device
    out = torch.empty_like(g) if out is None else out
    _need_out(out, "out", torch.float64, (R, n), dev)
    ws = _workspace(OP_MLL_ADJOINT, kd, R, m, F64, dev, ws)
    _check(lib().ldk_mll_adjoint(kd, R, m, _ptr(g), _ptr(out), _ptr(ws), _stream()),
           "ldk_mll_adjoint")
    return out


def kernel_grad(k: Kernel, ps: PointSet, n_min: int, n_max: int, a: torch.Tensor, pts=None,
                x0=None, dtype=torch.float64, out=None, ws=None, k1=None):
    """[R][d + 1]: sum_i a_i dk1_i/dlog gamma_j (j < d) and sum_i a_i k1_i (log zeta).
    k1: optionally the forward column of the same arguments and dtype (one
    sweep over the dimensions instead of two)."""
    dt = _dtype_code(dtype)
    dev = _dev_of(ps)
    _need_f64(a, "a", (ps.R, n_max - n_min), dev)
    if out is None:
        out = torch.empty((ps.R, ps.d + 1), dtype=torch.float64, device=dev)
    _need_out(out, "out", torch.float64, (ps.R, ps.d + 1), dev)
    if pts is not None:
        _need_out(pts, "pts", torch.int64, (ps.R, n_max - n_min, ps.d), dev)
    if x0 is not None:
        _need_out(x0, "x0", torch.int64, (ps.R, ps.d), dev)
    ws = _need_ws(ws, lib().ldk_kernel_grad_workspace_bytes(ps.R, ps.d, n_min, n_max,
                                                            int(pts is not None)), dev)
    if k1 is not None:
        _need_out(k1, "k1", _real(dt), (ps.R, n_max - n_min), dev)
    _check(lib().ldk_kernel_grad(C.byref(_k_checked(k, ps.d, dev)), C.byref(_ps_checked(ps)),
                                 _ptr(pts), _ptr(x0), n_min, n_max, dt, _ptr(k1), _ptr(a),
                                 _ptr(out), _ptr(ws), _stream()), "ldk_kernel_grad")
    return out


def fwht_split16(x: torch.Tensor, out=None):
    """Orthonormal FWHT of float32 rows on the matrix cores (split FP16)."""
    _need(x, "x")
    if x.dtype != torch.float32:
        raise LdkError("fwht_split16 takes float32 rows")
    n = x.shape[-1]
    m = _m_of(n)
    B = x.numel() // n
    out = torch.empty_like(x) if out is None else out
    _need_out(out, "out", torch.float32, x.shape, x.device)
    _check(lib().ldk_fwht_split16(B, m, _ptr(x), _ptr(out), _stream()), "ldk_fwht_split16")
    return out
