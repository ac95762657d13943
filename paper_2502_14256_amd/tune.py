"""Tuner of the transform plans (tile size, butterfly radix and, for FP32
digital-net rows of 2^12 and more, the engine: FP32 butterflies or the
split-FP16 matrix-core passes).

For each case (kind, working dtype, log2 n, rows, op) it loads, one at a
time, a one-entry table for every candidate (log_tile, radix, engine) that
the library accepts, times the op captured in a HIP graph and replayed K
times, and keeps the fastest.  The chosen entries are written in the format
ldk_init_tuned reads; every timing is returned too.

Run on the GPU the table is for:
    python -m paper_2502_14256_amd.tune --out paper_2502_14256_amd/tuned_mi355x.txt
"""
from __future__ import annotations

import argparse
import math
import os
import tempfile

import numpy as np
import torch

import paper_2502_14256_amd as ldk

LOG_TILES = (9, 10, 11, 12)
LOG_RADIX = (2, 3)
KINDS = {"lattice": ldk.LATTICE, "dnet": ldk.DNET_B2}


def default_cases():
    """The shapes the benchmark and the workloads run: single solves and
    16-column solves at n = 2^20, the fit of one column and one response,
    the batched table's groups (about 18 instances of 8 right-hand sides per
    (kind, size), n = 2^12 .. 2^18) and the gradient workload's eigenvalues
    (64 rows of 2^16)."""
    cases = []
    for kind in ("lattice", "dnet"):
        for rows in (1, 16):
            cases.append((kind, ldk.F64, 20, rows, "solve"))
        for m in range(12, 19):
            cases.append((kind, ldk.F64, m, 144, "solve"))
            cases.append((kind, ldk.F64, m, 18, "eig"))
    cases.append(("lattice", ldk.F64, 20, 2, "fit"))
    cases.append(("dnet", ldk.F64, 16, 64, "eig"))
    # FP32 nets: the same solve shapes, and the gradient workload's
    # likelihood (64 rows of 2^16)
    for rows in (1, 16):
        cases.append(("dnet", ldk.F32, 20, rows, "solve"))
    for m in range(12, 19):
        cases.append(("dnet", ldk.F32, m, 144, "solve"))
    cases.append(("dnet", ldk.F32, 16, 64, "mll"))
    return cases


def _time(fn, K):
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(K):
        g.replay()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / K


def _op(kind, dtype, m, rows, op, seed=0):
    """A closure running `op` once on synthetic data of the case's shape."""
    rng = np.random.default_rng(seed)
    n = 2 ** m
    dt = torch.float64 if dtype == ldk.F64 else torch.float32
    kd = KINDS[kind]
    if op == "solve":
        lam = torch.from_numpy(1.0 + rng.random((1, n))).cuda()
        y = torch.from_numpy(rng.standard_normal((1, rows, n))).to(dt).cuda()
        c = torch.empty_like(y)
        ws = ldk._workspace(ldk.OP_SOLVE, kd, rows, m, dtype, "cuda")
        return lambda: ldk.solve(kind, lam, 1e-3, y, out=c, ws=ws)
    if op == "eig":
        k1 = torch.from_numpy(rng.standard_normal((rows, n))).to(dt).cuda()
        lam = torch.empty((rows, n), dtype=torch.float64, device="cuda")
        ws = ldk._workspace(ldk.OP_EIG, kd, rows, m, dtype, "cuda")
        return lambda: ldk.eig(kind, k1, out=lam, ws=ws)
    if op == "fit":
        # rows = R (nrhs + 1) with one response per column
        R = max(rows // 2, 1)
        k1 = torch.from_numpy(1.0 + 0.1 * rng.standard_normal((R, n))).to(dt).cuda()
        y = torch.from_numpy(rng.standard_normal((R, 1, n))).to(dt).cuda()
        lam = torch.empty((R, n), dtype=torch.float64, device="cuda")
        c = torch.empty_like(y)
        ld = torch.empty(R, dtype=torch.float64, device="cuda")
        ws = ldk._workspace(ldk.OP_FIT, kd, 2 * R, m, dtype, "cuda")
        return lambda: ldk.fit(kind, k1, 1e-3, y, lam=lam, c=c, logdet=ld, ws=ws)
    if op == "mll":
        lam = torch.from_numpy(1.0 + rng.random((rows, n))).cuda()
        y = torch.from_numpy(rng.standard_normal((rows, n))).to(dt).cuda()
        g = torch.empty((rows, n), dtype=torch.float64, device="cuda")
        ws = ldk._workspace(ldk.OP_MLL, kd, rows, m, dtype, "cuda")
        return lambda: ldk.mll(kind, lam, 1e-3, y, out_g=g, ws=ws)
    raise ValueError(op)


def _table_line(kind, dtype, m, rows, log_tile, log_radix, engine=0):
    return f"{KINDS[kind]} {dtype} {m} {int(math.log2(rows))} {log_tile} {log_radix} {engine}\n"


def tune(cases=None, K: int = 20, out: str | None = None, verbose: bool = True):
    """Time every accepted candidate for every case; write the fastest to
    `out` (when given).  Returns [(case, [(log_tile, log_radix, engine, ms)],
    best)]."""
    ldk.init()
    cases = cases or default_cases()
    results, lines = [], []
    tmpdir = tempfile.mkdtemp(prefix="ldk_tune_")
    path = os.path.join(tmpdir, "candidate.txt")
    def load(entries):
        with open(path, "w") as f:
            f.writelines(_table_line(kind, dtype, m, rows, *e) for e in entries)
        ldk.load_tuned(path)

    for case in cases:
        kind, dtype, m, rows, op = case
        accepted = []
        cands = [(lt, lr, 0) for lt in LOG_TILES for lr in LOG_RADIX]
        if kind == "dnet" and dtype == ldk.F32 and m >= 12:
            cands.append((12, 3, 1))  # the matrix-core passes (tile and radix unused)
        for e in cands:
            try:
                load([e])
                accepted.append(e)
            except ldk.LdkError:
                pass  # a plan the pass kernels cannot run
        # workspaces sized while every candidate is in the table (the size
        # covers every plan the table may select), then one candidate at a time
        load(accepted)
        fn = _op(kind, dtype, m, rows, op)
        timings = []
        for e in accepted:
            load([e])
            timings.append((*e, _time(fn, K)))
        ldk.load_tuned(None)
        best = min(timings, key=lambda t: t[3])
        lines.append(_table_line(kind, dtype, m, rows, best[0], best[1], best[2]))
        results.append((case, timings, best))
        if verbose:
            dflt = ldk.plan_info(kind, dtype, m, rows)
            t_dflt = dict(((t[0], t[1], t[2]), t[3]) for t in timings).get(
                (dflt["log_tile"], 3, 0), float("nan"))
            what = "split16 matrix cores" if best[2] else f"tile 2^{best[0]} radix {2 ** best[1]}"
            print(f"{kind:8s} dtype={dtype} m={m:2d} rows={rows:4d} {op:5s}: best {what} "
                  f"{best[3] * 1e3:8.2f} us (default tile 2^{dflt['log_tile']}: "
                  f"{t_dflt * 1e3:8.2f} us)", flush=True)
        del fn
    if out:
        with open(out, "w") as f:
            f.write("# kind dtype m rows_log2 log_tile log2_radix engine  (ldk_init_tuned; "
                    "written by paper_2502_14256_amd/tune.py)\n")
            f.writelines(lines)
    return results


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--out", default=None)
    p.add_argument("--steps", type=int, default=20)
    a = p.parse_args()
    torch.cuda.set_device(0)
    tune(K=a.steps, out=a.out)


if __name__ == "__main__":
    main()
