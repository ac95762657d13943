"""Batched fit of an instance table of mixed kind and size, through the
library's batch plan (ldk_plan_create / ldk_plan_bind / ldk_batch_launch /
ldk_batch_capture).

An instance is one randomized point set (a rank-1 lattice or a base-2 net,
one shared generating vector or matrix per kind, a scramble and shift of its
own) with n = 2^m points and nrhs responses.  The plan groups the table by
(kind, m, nrhs): a group's instances are the replications of one point set,
so each group is one first-column launch and one fit (eigenvalues, every
solve and the log-det), and groups are shared out over the plan's streams.
Captured once, the whole table replays as one HIP graph.

This module only arranges the arenas the plan lays out (torch tensors) and
issues library calls; every step of the computation runs in the library's
kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import (DNET_B2, LATTICE, OP_EIG, OP_LOGDET, OP_SOLVE, Kernel, LdkError, PointSet,
               _Kernel, _check, _dtype_code, _kind, _stream, _workspace, eig, kernel_column, lib,
               logdet, solve)

ARENA_Y, ARENA_C, ARENA_LAM, ARENA_LOGDET, ARENA_WS, ARENA_K1 = 0, 1, 2, 3, 4, 5


class _BatchDesc(C.Structure):
    _fields_ = [("d", C.c_int32), ("m_max", C.c_int32), ("dtype", C.c_int32),
                ("streams", C.c_int32), ("sigma2", C.c_double), ("lattice_gen", C.c_void_p),
                ("net_gen", C.c_void_p), ("lattice_kernel", _Kernel), ("net_kernel", _Kernel)]


class _Instance(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("nrhs", C.c_int32),
                ("reserved", C.c_int32), ("shift", C.c_void_p), ("lms", C.c_void_p)]


def _dev_u64(a) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64).copy()).cuda()


@dataclass
class Instance:
    """One problem of the table (host arrays).

    kind: "lattice" or "dnet"; m: log2 of the point count; shift: uint64[d];
    lms: uint64[d][64] for nets (None for none); y: float[nrhs][2^m]."""

    kind: str
    m: int
    shift: np.ndarray
    y: np.ndarray
    lms: np.ndarray | None = None


_SIGS = {
    "ldk_plan_create": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "ldk_plan_arena_bytes": ([C.c_void_p, C.c_int], C.c_size_t),
    "ldk_plan_instance_offset": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "ldk_plan_bind": ([C.c_void_p] * 6 + [C.c_void_p], C.c_int),
    "ldk_batch_launch": ([C.c_void_p, C.c_void_p], C.c_int),
    "ldk_batch_capture": ([C.c_void_p, C.c_void_p], C.c_int),
    "ldk_plan_stats": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "ldk_plan_destroy": ([C.c_void_p], C.c_int),
}


def _L():
    L = lib()
    if not getattr(L, "_batch_sigs", False):
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        L._batch_sigs = True
    return L


class BatchFit:
    """Fit (first column, eigenvalues, solves, log-det) of every instance.

    gen: {"lattice": g[d], "dnet": C[d][m_max]} shared generators;
    alpha: the orders (one sequence for both kinds, or {"lattice": ..., "dnet":
    ...}); gamma, zeta: the product weights; sigma2: the nugget; streams:
    the plan's streams (1..8)."""

    def __init__(self, instances, gen: dict, m_max: int, alpha, gamma, zeta: float,
                 sigma2: float, dtype=torch.float64, streams: int = 1):
        if not instances:
            raise LdkError("empty instance table")
        L = _L()
        self.n_inst = len(instances)
        self.dtype = dtype
        self.sigma2 = float(sigma2)
        d = len(instances[0].shift)
        self.d, self.m_max = d, m_max
        alpha_of = alpha if isinstance(alpha, dict) else {"lattice": alpha, "dnet": alpha}
        self._gamma = torch.as_tensor(np.asarray(gamma, np.float64)).cuda()
        self._kern = {k: Kernel(k, np.asarray(alpha_of[k], np.int32), self._gamma, zeta)
                      for k in ("lattice", "dnet")}
        self._gen = {k: _dev_u64(gen[k]) for k in ("lattice", "dnet") if k in gen}
        self._inst = instances
        # per-instance device copies the plan gathers at bind
        self._shift = [_dev_u64(ins.shift) for ins in instances]
        self._lms = [None if ins.lms is None else _dev_u64(ins.lms) for ins in instances]
        arr = (_Instance * self.n_inst)()
        for i, ins in enumerate(instances):
            arr[i] = _Instance(_kind(ins.kind), int(ins.m), int(ins.y.shape[0]), 0,
                               self._shift[i].data_ptr(),
                               None if self._lms[i] is None else self._lms[i].data_ptr())
        self._desc = _BatchDesc(d, m_max, _dtype_code(dtype), int(streams), self.sigma2,
                                self._gen["lattice"].data_ptr() if "lattice" in self._gen else None,
                                self._gen["dnet"].data_ptr() if "dnet" in self._gen else None,
                                self._kern["lattice"]._c(), self._kern["dnet"]._c())
        plan = C.c_void_p()
        _check(L.ldk_plan_create(C.byref(self._desc), self.n_inst, arr, C.byref(plan)),
               "ldk_plan_create")
        self._plan = plan
        nb = [int(L.ldk_plan_arena_bytes(plan, w)) for w in range(5)]
        self._y = torch.empty(max(nb[ARENA_Y], 1), dtype=torch.uint8, device="cuda").view(dtype)
        self._c = torch.empty(max(nb[ARENA_C], 1), dtype=torch.uint8, device="cuda").view(dtype)
        self._lam = torch.empty(max(nb[ARENA_LAM] // 8, 1), dtype=torch.float64, device="cuda")
        self._ld = torch.empty(max(nb[ARENA_LOGDET] // 8, 1), dtype=torch.float64, device="cuda")
        self._ws = torch.empty(max(nb[ARENA_WS], 256), dtype=torch.uint8, device="cuda")
        self.arena_bytes = dict(zip(("y", "c", "lam", "logdet", "ws"), nb))
        # responses into their rows
        for i, ins in enumerate(instances):
            self.y(i).copy_(torch.from_numpy(np.ascontiguousarray(ins.y)).to(dtype))
        _check(L.ldk_plan_bind(plan, self._y.data_ptr(), self._c.data_ptr(),
                               self._lam.data_ptr(), self._ld.data_ptr(), self._ws.data_ptr(),
                               _stream()), "ldk_plan_bind")
        g = C.c_int()
        _check(L.ldk_plan_stats(plan, C.byref(g), None), "ldk_plan_stats")
        self.n_groups = g.value

    # ---- views into the arenas -------------------------------------------
    def _off(self, i, which):
        o = C.c_size_t()
        _check(_L().ldk_plan_instance_offset(self._plan, i, which, C.byref(o)),
               "ldk_plan_instance_offset")
        return o.value

    def _shape(self, i):
        ins = self._inst[i]
        return int(ins.y.shape[0]), 2 ** int(ins.m)

    def y(self, i):
        nrhs, n = self._shape(i)
        o = self._off(i, ARENA_Y)
        return self._y[o:o + nrhs * n].view(nrhs, n)

    def c(self, i):
        nrhs, n = self._shape(i)
        o = self._off(i, ARENA_C)
        return self._c[o:o + nrhs * n].view(nrhs, n)

    def lam(self, i):
        _, n = self._shape(i)
        o = self._off(i, ARENA_LAM)
        return self._lam[o:o + n]

    def logdet(self, i):
        o = self._off(i, ARENA_LOGDET)
        return self._ld[o]

    def k1(self, i):
        """Instance i's first column (in the workspace arena)."""
        _, n = self._shape(i)
        o = self._off(i, ARENA_K1)
        return self._ws.view(self.dtype)[o:o + n]

    def result(self, i):
        """(c[nrhs][n], log-det) of instance i, as device views."""
        return self.c(i), self.logdet(i)

    # ---- execution ------------------------------------------------------------
    def step(self):
        """Enqueue the whole table on the current stream (replays the
        captured graph after capture())."""
        _check(_L().ldk_batch_launch(self._plan, _stream()), "ldk_batch_launch")

    def capture(self):
        """Capture the table's launches as one HIP graph kept by the plan
        (on a side stream: the null stream cannot be captured); later
        step() calls replay it."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            _check(_L().ldk_batch_capture(self._plan, _stream()), "ldk_batch_capture")
        torch.cuda.current_stream().wait_stream(s)
        return self

    def kernel_nodes(self) -> int:
        k = C.c_int()
        _check(_L().ldk_plan_stats(self._plan, None, C.byref(k)), "ldk_plan_stats")
        return k.value

    def step_plain(self):
        """The same work issued instance by instance with the separate entry
        points (first column, eigenvalues, solve, log-det of one instance per
        call), into the same arenas: the unbatched reference."""
        if not hasattr(self, "_plain"):
            self._plain = []
            for i, ins in enumerate(self._inst):
                kd, dt = _kind(ins.kind), _dtype_code(self.dtype)
                nrhs, n = self._shape(i)
                m = int(ins.m)
                gen = self._gen[ins.kind]
                lms = self._lms[i]
                ps = PointSet(ins.kind, 1, self.d, self.m_max, gen,
                              None if lms is None else lms.view(1, self.d, 64),
                              self._shift[i].view(1, self.d))
                k1 = torch.empty((1, n), dtype=self.dtype, device="cuda")
                ws = dict(eig=_workspace(OP_EIG, kd, 1, m, dt, "cuda"),
                          solve=_workspace(OP_SOLVE, kd, nrhs, m, dt, "cuda"),
                          ld=_workspace(OP_LOGDET, kd, 1, m, dt, "cuda"))
                self._plain.append((i, ins.kind, ps, k1, ws, n))
        for i, kind, ps, k1, ws, n in self._plain:
            kernel_column(self._kern[kind], ps, 0, n, dtype=self.dtype, out=k1)
            lam = self.lam(i).view(1, n)
            eig(kind, k1, out=lam, ws=ws["eig"])
            solve(kind, lam, self.sigma2, self.y(i)[None], out=self.c(i)[None], ws=ws["solve"])
            logdet(lam, self.sigma2, out=self._ld[self._off(i, ARENA_LOGDET):][:1],
                   ws=ws["ld"])

    def __del__(self):
        try:
            if getattr(self, "_plan", None):
                torch.cuda.synchronize()
                _L().ldk_plan_destroy(self._plan)
                self._plan = None
        except Exception:
            pass
