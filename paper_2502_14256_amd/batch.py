"""Batched fit over an instance table of mixed kind and size.

An instance is one randomized point set with its own responses: a rank-1
lattice or a base-2 net (one shared generating vector or matrix per kind, a
scramble and shift of its own), n = 2^m points, nrhs responses.  Solving
instance after instance launches every op once per instance, and at n = 2^12
one launch is a few workgroups.  Here instances of the same kind and size
are the replications of one point set (Sec. 4: R independent randomizations
of one sequence), so each op runs once per (kind, m) group over all its
instances: the first column (points regenerated in registers), the
eigenvalues, the solve of every right-hand side and the log-det.  All the
groups' launches are enqueued on one stream and can be captured as one HIP
graph (`capture`), which replays the whole table with one host call.

This module only arranges buffers and issues library calls; every step of
the computation runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import (LdkError, Kernel, OP_EIG, OP_FIT, OP_LOGDET, OP_SOLVE, PointSet, _dtype_code,
               _kind, _workspace, eig, fit, interlace, kernel_column, logdet, solve)


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


class BatchFit:
    """Fit (first column, eigenvalues, solves, log-det) of every instance.

    gen: {"lattice": g[d], "dnet": C[d][m_max]} shared generators;
    alpha, gamma, zeta: the product kernel per kind ({"lattice": ..., "dnet": ...}
    for alpha, or one sequence for both), sigma2: the nugget."""

    def __init__(self, instances, gen: dict, m_max: int, alpha, gamma, zeta: float,
                 sigma2: float, dtype=torch.float64):
        if not instances:
            raise LdkError("empty instance table")
        self.n_inst = len(instances)
        self.sigma2 = float(sigma2)
        self.dtype = dtype
        d = len(instances[0].shift)
        nrhs = instances[0].y.shape[0]
        self.nrhs = nrhs
        keys = sorted({(ins.kind, ins.m) for ins in instances})
        self.groups = []
        # (group index, row) of every instance, in table order
        self.where = [None] * self.n_inst
        alpha_of = alpha if isinstance(alpha, dict) else {"lattice": alpha, "dnet": alpha}
        gamma_d = torch.as_tensor(np.asarray(gamma, np.float64)).cuda()
        for gi, (kind, m) in enumerate(keys):
            members = [i for i, ins in enumerate(instances) if ins.kind == kind and ins.m == m]
            R, n = len(members), 2 ** m
            shift = np.stack([instances[i].shift for i in members])
            lms = None
            if kind == "dnet" and instances[members[0]].lms is not None:
                lms = np.stack([instances[i].lms for i in members])
            ps = PointSet(kind, R, d, m_max, _dev_u64(gen[kind]),
                          None if lms is None else _dev_u64(lms), _dev_u64(shift))
            if lms is not None and m_max > 0:
                # each instance's scrambled columns S_j C_j, formed once with
                # the plan (interlacing of order 1): the same points, and the
                # column kernel no longer scrambles in every block
                ps = interlace(ps, 1, shift=ps.shift)
            kern = Kernel(kind, np.asarray(alpha_of[kind], np.int32), gamma_d, zeta)
            y = torch.from_numpy(np.ascontiguousarray(
                np.stack([instances[i].y for i in members]))).to(device="cuda", dtype=dtype)
            if y.shape != (R, nrhs, n):
                raise LdkError("every instance needs nrhs x 2^m responses")
            kd, dt = _kind(kind), _dtype_code(dtype)
            g = dict(kind=kind, m=m, n=n, R=R, members=members, ps=ps, kern=kern, y=y,
                     k1=torch.empty((R, n), dtype=dtype, device="cuda"),
                     lam=torch.empty((R, n), dtype=torch.float64, device="cuda"),
                     c=torch.empty_like(y),
                     ld=torch.empty(R, dtype=torch.float64, device="cuda"),
                     ws_fit=_workspace(OP_FIT, kd, R * (nrhs + 1), m, dt, "cuda"))
            for row, i in enumerate(members):
                self.where[i] = (gi, row)
            self.groups.append(g)
        self.graph = None

    def step(self):
        """Enqueue the whole table on the current stream: per group, the
        first column, then eigenvalues, solves and log-det in one fit call."""
        for g in self.groups:
            kernel_column(g["kern"], g["ps"], 0, g["n"], dtype=self.dtype, out=g["k1"])
            fit(g["kind"], g["k1"], self.sigma2, g["y"], lam=g["lam"], c=g["c"], logdet=g["ld"],
                ws=g["ws_fit"])

    def step_plain(self):
        """The same work issued instance by instance with the separate entry
        points (one launch of every op per instance, on row views of the same
        buffers): the unbatched reference the batched step is compared with."""
        if not hasattr(self, "_plain"):
            self._plain = []
            for g in self.groups:
                kd, dt = _kind(g["kind"]), _dtype_code(self.dtype)
                ws = dict(eig=_workspace(OP_EIG, kd, 1, g["m"], dt, "cuda"),
                          solve=_workspace(OP_SOLVE, kd, self.nrhs, g["m"], dt, "cuda"),
                          ld=_workspace(OP_LOGDET, kd, 1, g["m"], dt, "cuda"))
                ps = g["ps"]
                for row in range(g["R"]):
                    sl = slice(row, row + 1)
                    psr = PointSet(g["kind"], 1, ps.d, ps.m_max,
                                   ps.gen[sl] if ps.per_replication else ps.gen,
                                   None if ps.lms is None else ps.lms[sl], ps.shift[sl],
                                   per_replication=ps.per_replication)
                    self._plain.append((g, sl, psr, ws))
        for g, sl, psr, ws in self._plain:
            kernel_column(g["kern"], psr, 0, g["n"], dtype=self.dtype, out=g["k1"][sl])
            eig(g["kind"], g["k1"][sl], out=g["lam"][sl], ws=ws["eig"])
            solve(g["kind"], g["lam"][sl], self.sigma2, g["y"][sl], out=g["c"][sl], ws=ws["solve"])
            logdet(g["lam"][sl], self.sigma2, out=g["ld"][sl], ws=ws["ld"])

    def capture(self, plain: bool = False) -> torch.cuda.CUDAGraph:
        """Capture step() (or step_plain()) as one HIP graph, after one eager run."""
        fn = self.step_plain if plain else self.step
        fn()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fn()
        if not plain:
            self.graph = graph
        return graph

    def result(self, i: int):
        """(c[nrhs][n], log-det) of instance i, as device views."""
        gi, row = self.where[i]
        g = self.groups[gi]
        return g["c"][row], g["ld"][row]
