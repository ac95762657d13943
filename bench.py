"""Benchmark of the fast kernel-method hot path on one MI355X.

A step is one pass of the whole path over the rank-1 lattice workload
(n = 2^20, d = 32, order-2 SI kernel, gamma_j = 1/j^2, sigma^2 = 1e-3):
  points + first column in one call (points_column: the point words and
  k1, the column regenerating the points in registers) -> fit (eig (FFTBR),
  solve, logdet in one call),
with the generating vector, shift and responses already resident in HBM.
The metric counts one Gram solve (K + sigma^2 I)^-1 y per step: `value` is
whole steps per second (each step also forms the points, the first column,
the eigenvalues and the log-det); `solves_per_s_cached_lambda` is the solve
alone.

Printed: one JSON line with
- the metric and per-op timings (HIP events on the library's stream);
- `roofline`: the Gram solve with cached eigenvalues (the metric's target),
  and the step's longest single kernel (the point writer) beside it;
- `solve_rhs`: solves with 1 and 16 right-hand sides at n = 2^20 (lattice
  and net), solves/s and fraction of the HBM peak;
- `fp32_step` (the same step with FP32 responses and solve) and
  `c1_latency` (the small net problem end to end);
- the marginal-likelihood gradient workload (64 replications of a net with
  n = 2^16, d = 64) under "grad", and the batched instance table under
  "batched";
- the split-FP16 matrix-core FWHT ("fwht_split16"), the higher-order net
  ("higher_order_net"), kernel cubature ("cubature"), the RQMC estimate
  ("rqmc"), and the doubling update ("update_double");
- the CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# transform plans chosen by paper_2502_14256_amd/tune.py on an MI355X
TUNED_TABLE = os.path.join(ROOT, "paper_2502_14256_amd", "tuned_mi355x.txt")

# HBM bytes per call, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of the
# graph-free probes (`bench.py --traffic-probe`: the points + column kernel
# k_points_kcol_lattice at n = 2^20, d = 32; `bench.py --solve-probe`: the
# three kernels of one FP64 lattice solve at n = 2^20, one RHS), each scaled
# by the counters of a plain device copy of known size in the same program
# (x2 reads, x1 writes; profiles/traffic_lattice_m20_d32_f64.md).  Valid only
# for the kernel sources they were taken on: the sources' SHA-1 is checked at
# run time and the figure reported as null once they change.
STEP_TRAFFIC = {"read_MiB": 0.21, "write_MiB": 264.00,
                "sources": ('kcol.hip', 'kfactor.hpp', 'pointset.hpp', 'common.hpp'),
                "sha1": "88f23a88bafdd2984406a1f7a66de15a4370acf2"}
SOLVE_TRAFFIC = {"read_MiB": 34.33, "write_MiB": 24.06,
                 "sources": ('transform.hip', 'realfft.hip', 'passkit.hpp', 'transform.hpp', 'common.hpp'),
                 "sha1": "ef2fd51aed0b23c8e166cde8b2a124cbd6c938a5"}


def traffic_bytes(rec):
    import hashlib

    if rec["sha1"] is None:
        return None
    h = hashlib.sha1()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2502_14256_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sha1"]:
        return None
    return int((rec["read_MiB"] + rec["write_MiB"]) * 2**20)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--dtype", choices=["f64", "f32"], default="f64",
                   help="arithmetic of the first column and the per-solve data (y, c, solve "
                        "transforms); the eigenvalues, division and log-det stay FP64")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-tuned", action="store_true",
                   help="use the default transform plans, not the tuned table "
                        "(paper_2502_14256_amd/tuned_mi355x.txt)")
    p.add_argument("--no-grad", action="store_true",
                   help="skip the marginal-likelihood gradient workload")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the batched instance-table workload")
    p.add_argument("--batch-steps", type=int, default=10)
    p.add_argument("--traffic-probe", action="store_true",
                   help="only run the step eagerly 5 times and a 256 MiB device copy 5 times "
                        "(a short program for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs; the "
                        "copy calibrates the counters), then exit")
    p.add_argument("--solve-probe", action="store_true",
                   help="only run the cached-lambda Gram solve (lattice n=2^20, FP64, 1 RHS) 20 "
                        "times eagerly, then a 32 MiB device copy 5 times (a short graph-free "
                        "program for rocprofv3 kernel traces and FETCH_SIZE / WRITE_SIZE runs; "
                        "the copy calibrates the counters), then exit")
    p.add_argument("--valu-probe", action="store_true",
                   help="only run the step, the FP32 gradient step, the RQMC estimates and the structure-free generators a few "
                        "times (a short program for rocprofv3 --pmc SQ_INSTS_VALU runs), then exit")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path "
              "(independent replications would shard with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    torch.cuda.set_device(0)
    tuned = None if args.no_tuned else TUNED_TABLE
    if tuned is not None and not os.path.exists(tuned):
        tuned = None
    global _TUNED_PATH
    _TUNED_PATH = tuned
    ldk.init(tuned=tuned)
    dt = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if args.dtype == "f64" else 4

    w = W.workload(2)
    n, d, R, m = 2 ** w["m"], w["d"], w["R"], w["m"]

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps = ldk.PointSet("lattice", R, d, m, dev_u64(w["gen"]), None, dev_u64(w["shift"]))
    kern = ldk.Kernel("lattice", w["alpha"],
                      torch.tensor(w["gamma"], dtype=torch.float64, device="cuda"), w["zeta"])
    # responses y = sum_j sin(2 pi x_j)/j + noise at the points (input synthesis, untimed)
    pts0 = ldk.gen_points(ps, 0, n)
    x = W.to_unit_f64(pts0.cpu().numpy().view(np.uint64))
    y_host = np.ascontiguousarray(W.sine_response(x, w["eps"][:, 0, :])[:, None, :])
    del pts0, x
    y = torch.from_numpy(y_host).to(device="cuda", dtype=dt)

    # outputs and workspaces, allocated once
    pts = torch.empty((R, n, d), dtype=torch.int64, device="cuda")
    k1 = torch.empty((R, n), dtype=dt, device="cuda")
    lam = torch.empty((R, n), dtype=torch.float64, device="cuda")
    c = torch.empty_like(y)
    ld = torch.empty(R, dtype=torch.float64, device="cuda")
    ws_solve = ldk._workspace(ldk.OP_SOLVE, ldk.LATTICE, R, m, ldk._dtype_code(dt), "cuda")
    ws_ld = ldk._workspace(ldk.OP_LOGDET, ldk.LATTICE, R, m, ldk.F64, "cuda")
    ws_eig = ldk._workspace(ldk.OP_EIG, ldk.LATTICE, R, m, ldk._dtype_code(dt), "cuda")
    ws_fit = ldk._workspace(ldk.OP_FIT, ldk.LATTICE, R * 2, m, ldk._dtype_code(dt), "cuda")

    ops = ["points_column", "fit"]

    def step():
        # point words and first column in one launch (the column regenerates
        # the points in registers, so the two run side by side)
        ldk.points_column(kern, ps, 0, n, dtype=dt, pts=pts, k1=k1)
        # eigenvalues, solve and log-det in one call (shared tile passes)
        ldk.fit("lattice", k1, w["sigma2"], y, lam=lam, c=c, logdet=ld, ws=ws_fit)

    if args.valu_probe:
        for _ in range(3):
            step()
        grad_bench(2, 1, probe=True)
        rqmc_bench(3, probe=True)
        structure_free_probe()
        torch.cuda.synchronize()
        print(json.dumps({"valu_probe": True}), flush=True)
        return

    if args.solve_probe:
        # eigenvalues once (untimed), then the solve alone, no graphs
        ldk.points_column(kern, ps, 0, n, dtype=dt, pts=pts, k1=k1)
        ldk.eig("lattice", k1, out=lam, ws=ws_eig)
        for _ in range(20):
            ldk.solve("lattice", lam, w["sigma2"], y, out=c, ws=ws_solve)
        src = torch.empty(4 * 2**20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"solve_probe": True, "copy_bytes": src.numel() * 8}), flush=True)
        return

    if args.traffic_probe:
        for _ in range(5):
            step()
        src = torch.empty(32 * 2**20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": src.numel() * 8}), flush=True)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    c_eager, ld_eager, pts_eager = c.clone(), ld.clone(), pts.clone()

    # One whole step captured as a HIP graph: replays carry no host launch
    # overhead.  Every library call enqueues on torch's current stream, which
    # is the capture stream inside the context; no allocation or memset is
    # captured (all buffers and workspaces exist already).  (Putting the
    # point words on a second stream beside the rest was measured: the
    # hardware does not overlap the two, so the step stays one stream.)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    graph_matches = bool(torch.equal(c, c_eager) and torch.equal(ld, ld_eager)
                         and torch.equal(pts, pts_eager))

    # timed region 1: K whole steps (graph replays), HIP events on the stream
    K = args.steps
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(K):
        graph.replay()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)

    # timed region 2: each op alone, captured in its own graph and replayed K
    # times back to back (device time per launch, no host gaps)
    op_calls = {
        "points_column": lambda: ldk.points_column(kern, ps, 0, n, dtype=dt, pts=pts, k1=k1),
        "gen_points": lambda: ldk.gen_points(ps, 0, n, out=pts),
        "kernel_column": lambda: ldk.kernel_column(kern, ps, 0, n, dtype=dt, out=k1),
        "fit": lambda: ldk.fit("lattice", k1, w["sigma2"], y, lam=lam, c=c, logdet=ld, ws=ws_fit),
        "eig": lambda: ldk.eig("lattice", k1, out=lam, ws=ws_eig),
        "solve": lambda: ldk.solve("lattice", lam, w["sigma2"], y, out=c, ws=ws_solve),
        "logdet": lambda: ldk.logdet(lam, w["sigma2"], out=ld, ws=ws_ld),
    }
    per_op = {op: time_graph(op_calls[op], K) for op in ops}
    # the separate entry points the fused calls replace, timed alone
    unfused = {op: round(time_graph(op_calls[op], K), 5)
               for op in ("gen_points", "kernel_column", "eig", "solve", "logdet")}
    # algorithmic bytes per op (one launch of each op per step)
    alg = {
        "points_column": (8 * d + esz) * n * R,   # write the point words and k1
        "gen_points": 8 * n * d * R,              # write the point words
        "kernel_column": esz * n * R,             # write k1 (points regenerated in registers)
        "fit": (3 * esz + 8) * n * R,             # read k1 and y, write lambda (FP64) and c
        "eig": (esz + 8) * n * R,                 # read k1, write lambda (FP64)
        "solve": (2 * esz + 8) * n * R,           # read y, read lambda (FP64), write c
        "logdet": 8 * n * R,                      # read lambda
    }
    op_rows = {op: {"ms": round(per_op[op], 5),
                    "alg_bytes": alg[op],
                    "GB_s": round(alg[op] / (per_op[op] * 1e-3) / 1e9, 1),
                    "hbm_frac": round(alg[op] / (per_op[op] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
               for op in ops}
    # the median and minimum over runs of graph replays, and the fractions
    # against a measured device copy rate beside those against 8 TB/s
    copy_gbs = copy_bandwidth(K)
    stats = {"step_ms": time_graph_stats(step, K), "solve_ms": time_graph_stats(op_calls["solve"], K),
             "fit_ms": time_graph_stats(op_calls["fit"], K),
             "copy_GB_s": copy_gbs,
             "note": "each: 5 runs of K graph replays after 3 warm-up replays; median and min of the "
                     "per-run means; copy_GB_s: a 256 MiB device copy (bytes read + written)"}
    # The headline roofline is the Gram solve with cached eigenvalues (the
    # target of the metric): read y and lambda, write c, 24 MiB at n = 2^20
    # in FP64, over the three kernels of one ldk_solve (row pass, top pass
    # with the filter, inverse row pass), captured alone in a graph: the
    # average launch over 5 runs of K replays (the mean of stats["solve_ms"]).
    # The step's longest single kernel is the point writer (points + first
    # column), reported separately.
    t_solve = stats["solve_ms"]["mean"]
    roof_dom = {"kernel": "ldk_solve, lattice n=2^20 FP64, 1 RHS, cached lambda (3 kernels: "
                          "row pass, top pass with the filter, inverse row pass)",
                "bound": "hbm",
                "achieved": round(alg["solve"] / (t_solve * 1e-3) / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(alg["solve"] / (t_solve * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": traffic_bytes(SOLVE_TRAFFIC)}
    roof_points = {"kernel": "k_points_kcol_lattice (points + first column; the step's longest "
                             "single kernel, not the solve)", "bound": "hbm",
                   "achieved": op_rows["points_column"]["GB_s"], "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": op_rows["points_column"]["hbm_frac"],
                   "traffic": traffic_bytes(STEP_TRAFFIC)}
    ms_per_step = total_ms / K
    solves_per_s = R * K / (total_ms * 1e-3)
    for r_ in (roof_dom, roof_points):
        r_["copy_GB_s"] = copy_gbs
        r_["frac_of_copy"] = round(r_["achieved"] / copy_gbs, 4)

    out = {
        "metric": "Gram solves/s and GB/s (% HBM peak) at n=2^20,d=32; batched+grad vs plain",
        "value": round(solves_per_s, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "lattice_m20_d32_si2 (rank-1 lattice n=2^20 d=32, order-2 SI "
                               "kernel, gamma_j=1/j^2, sigma^2=1e-3, one RHS): points + first "
                               "column (one call) + fit (eig, solve, logdet) per step",
                   "n": n, "d": d, "R": R, "nrhs": 1},
        "roofline": roof_dom,
        "step_longest_kernel_roofline": roof_points,
        "fit_roofline": {"bound": "hbm", "kernels": 3, "achieved": op_rows["fit"]["GB_s"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": op_rows["fit"]["hbm_frac"], "copy_GB_s": copy_gbs,
                         "frac_of_copy": round(op_rows["fit"]["GB_s"] / copy_gbs, 4)},
        "timing_stats": stats,
        "solves_per_s_cached_lambda": round(1e3 / t_solve, 1),
        "ops": op_rows,
        "unfused_ms": unfused,
        "timing": "value and ms_per_step: K replays of one HIP-graph-captured step; ops: each "
                  "op captured alone in a graph and replayed K times, HIP events around the "
                  "replays on the capture stream",
        "graph_equals_eager": graph_matches,
        "tuned_plans": os.path.relpath(tuned, ROOT) if tuned else None,
        "wall_s_timed": round(wall, 4),
    }

    out["solve_rhs"] = solve_rhs_bench(K, lam, w)
    if args.dtype == "f64":
        out["fp32_step"] = fp32_step_bench(K, kern, ps, w, y_host, c)
    out["c1_latency"] = c1_latency_bench(K)

    if not args.no_grad:
        out["grad"] = grad_bench(K, args.warmup)

    if not args.no_batch:
        out["batched"] = batch_bench(args.batch_steps, args.warmup)

    if "batched" in out and "grad" in out:
        bt, f, gr = out["batched"], out["batched"]["f32"], out["grad"]
        out["batched_mfma_grad_vs_plain"] = {
            "table_solves_per_s": {
                "batched_f32_split16_nets": f["batched_split16"]["solves_per_s"],
                "batched_f32_butterflies": f["batched_butterflies"]["solves_per_s"],
                "batched_f64": bt["value"],
                "plain_f32": f["plain_butterflies"]["solves_per_s"],
                "plain_f64": bt["plain_solves_per_s"]},
            "table_err_c_vs_f64_max": {
                "batched_f32_split16_nets": f["batched_split16"]["err_c_vs_f64_max"],
                "batched_f32_butterflies": f["batched_butterflies"]["err_c_vs_f64_max"],
                "plain_f32": f["plain_butterflies"]["err_c_vs_f64_max"]},
            "gradient_replications_per_s": {"batched_f32": gr["value"],
                                            "plain_f32": gr["plain_per_replication"]["value"]},
            "gradient_err_vs_f64": {"batched_f32": gr["f32_grad_rel_err_vs_f64"],
                                    "plain_f32": gr["plain_per_replication"]["grad_rel_err_vs_f64"]},
            "note": "the instance table (256 instances, n = 2^12..2^18, 8 RHS) and the gradient "
                    "workload (64 replications, n = 2^16, d = 64); FP32 errors against the "
                    "FP64 results of the same GPU path"}

    out["fwht_split16"] = fwht_bench(K)
    out["higher_order_net"] = higher_order_bench(K)
    out["cubature"] = cubature_bench(K, lam, y[:, 0, :], w)
    out["rqmc"] = rqmc_bench(K)
    out["update_double"] = update_bench(K)
    out["structure_free"] = structure_free_bench(K)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], c_oracle = cpu_baseline(w, y_host)
        # the step's result against the FP64 oracle (normwise), per dtype
        out["err_c_vs_fp64_oracle"] = {
            args.dtype: float(np.linalg.norm(c.double().cpu().numpy() - c_oracle)
                              / np.linalg.norm(c_oracle))}
        if "fp32_step" in out:
            out["err_c_vs_fp64_oracle"]["f32"] = float(
                np.linalg.norm(out["fp32_step"].pop("_c") - c_oracle) / np.linalg.norm(c_oracle))
    elif "fp32_step" in out:
        out["fp32_step"].pop("_c")

    print(json.dumps(out), flush=True)


_TUNED_PATH = None


def engine_table(engine):
    """A copy of the loaded tuned table in which every FP32 digital-net entry
    is replaced by one engine (0 FP32 butterflies, 1 split-FP16 matrix
    cores) for every m >= 12 and row count; returns its path."""
    import tempfile

    lines = []
    if _TUNED_PATH:
        with open(_TUNED_PATH) as f:
            lines = [ln for ln in f if not ln.split()[:2] == ["1", "1"]]
    lines += [f"1 1 {m} 0 12 3 {engine}\n" for m in range(12, 27)]
    fd, path = tempfile.mkstemp(prefix="ldk_engine_", suffix=".txt")
    with os.fdopen(fd, "w") as f:
        f.writelines(lines)
    return path


def with_engine(engine, fn):
    """fn() with the FP32 net engine forced; the tuned table afterwards."""
    import paper_2502_14256_amd as ldk

    path = engine_table(engine)
    try:
        ldk.load_tuned(path)
        return fn()
    finally:
        ldk.load_tuned(_TUNED_PATH)
        os.unlink(path)


def time_graph(fn, K):
    """Average device ms per launch of fn: captured once in a HIP graph, three
    warm-up replays, then the graph replayed K times between two events on
    the capture stream."""
    import torch

    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(K):
        g.replay()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / K


def time_graph_stats(fn, K, groups=5):
    """Device ms per launch of fn over `groups` runs of K graph replays each
    (after a warm-up replay), each run between two events on the capture
    stream: the mean over all runs, and the median and the minimum of the
    per-run means."""
    import statistics

    import torch

    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    runs = []
    for _ in range(groups):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(K):
            g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b) / K)
    return {"mean": round(sum(runs) / len(runs), 5), "median": round(statistics.median(runs), 5),
            "min": round(min(runs), 5), "runs": groups, "replays_per_run": K}


def copy_bandwidth(K):
    """Measured device copy rate (GB/s, bytes read + written): a 256 MiB
    device-to-device copy captured in a graph, median of the runs."""
    import torch

    src = torch.empty(32 * 2**20, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    st = time_graph_stats(lambda: dst.copy_(src), max(K // 5, 10))
    return round(2 * src.numel() * 8 / (st["median"] * 1e-3) / 1e9, 1)


def grad_bench(K, warmup, probe=False):
    """Marginal-likelihood gradient of the net workload: 64 replications of
    n = 2^16 points in d = 64 (LMS + digital shift, order-2 DSI kernel,
    gamma_j = 1/j^2, sigma^2 = 1e-3).  A step is the whole gradient for all
    replications: first column (FP32 factors, regenerated points) ->
    eigenvalues (FP64) -> likelihood and dL/dlambda (FP32 transform of y,
    FP64 after it) -> adjoint -> kernel-parameter gradient (FP32 factors,
    FP64 sums).  The FP32 gradient's error is measured against the same
    step in FP64."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    w = W.workload(5)
    m, d, R = w["m"], w["d"], w["R"]
    n = 2 ** m

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps = ldk.PointSet("dnet", R, d, m, dev_u64(w["gen"]), dev_u64(w["lms"]), dev_u64(w["shift"]))
    # each randomization's scrambled generating matrices S_j C_j, formed once
    # (interlacing of order 1): they do not change with the kernel
    # parameters, and the column and gradient kernels then read
    # per-replication columns instead of scrambling in every block
    ps = ldk.interlace(ps, 1, shift=ps.shift)
    kern = ldk.Kernel("dnet", w["alpha"],
                      torch.tensor(w["gamma"], dtype=torch.float64, device="cuda"), w["zeta"])
    y64 = torch.from_numpy(np.ascontiguousarray(w["y"][:, 0, :])).cuda()

    def buffers(dt):
        b = dict(k1=torch.empty((R, n), dtype=dt, device="cuda"),
                 lam=torch.empty((R, n), dtype=torch.float64, device="cuda"),
                 y=y64.to(dt),
                 g=torch.empty((R, n), dtype=torch.float64, device="cuda"),
                 a=torch.empty((R, n), dtype=torch.float64, device="cuda"),
                 kg=torch.empty((R, d + 1), dtype=torch.float64, device="cuda"),
                 L=torch.empty(R, dtype=torch.float64, device="cuda"),
                 ds=torch.empty(R, dtype=torch.float64, device="cuda"))
        code = ldk._dtype_code(dt)
        b["ws_eig"] = ldk._workspace(ldk.OP_EIG, ldk.DNET_B2, R, m, code, "cuda")
        b["ws_mll"] = ldk._workspace(ldk.OP_MLL, ldk.DNET_B2, R, m, code, "cuda")
        b["ws_grad"] = torch.empty(ldk.lib().ldk_kernel_grad_workspace_bytes(R, d, 0, n, 0),
                                   dtype=torch.uint8, device="cuda")
        return b

    def ops_of(b, dt):
        def mll():
            L, g, ds = b["L"], b["g"], b["ds"]
            code = ldk._dtype_code(dt)
            ldk._check(ldk.lib().ldk_mll(ldk.DNET_B2, R, m, code, ldk._ptr(b["lam"]), w["sigma2"],
                                         ldk._ptr(b["y"]), ldk._ptr(L), ldk._ptr(g), ldk._ptr(ds),
                                         ldk._ptr(b["ws_mll"]), ldk._stream()), "ldk_mll")
        return {
            "kernel_column": lambda: ldk.kernel_column(kern, ps, 0, n, dtype=dt, out=b["k1"]),
            "eig": lambda: ldk.eig("dnet", b["k1"], out=b["lam"], ws=b["ws_eig"]),
            "mll": mll,
            "mll_adjoint": lambda: ldk.mll_adjoint("dnet", b["g"], out=b["a"]),
            "kernel_grad": lambda: ldk.kernel_grad(kern, ps, 0, n, b["a"], dtype=dt, out=b["kg"],
                                                   ws=b["ws_grad"], k1=b["k1"]),
        }

    names = ["kernel_column", "eig", "mll", "mll_adjoint", "kernel_grad"]
    if probe:
        ops = ops_of(buffers(torch.float32), torch.float32)
        for _ in range(3):
            for nm in names:
                ops[nm]()
        return None

    def run(dt, per_op=True):
        b = buffers(dt)
        ops = ops_of(b, dt)

        def step():
            for nm in names:
                ops[nm]()

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ms = time_graph(step, K)
        grad = torch.cat([b["kg"], b["ds"][:, None]], dim=1).cpu().numpy()
        return dict(ms=ms, grad=grad, L=b["L"].cpu().numpy(),
                    per_op={nm: time_graph(ops[nm], K) for nm in names} if per_op else None)

    def run_plain(dt):
        # the unbatched form: the same calls one replication at a time
        b = buffers(dt)
        code = ldk._dtype_code(dt)
        ws_eig = ldk._workspace(ldk.OP_EIG, ldk.DNET_B2, 1, m, code, "cuda")
        ws_mll = ldk._workspace(ldk.OP_MLL, ldk.DNET_B2, 1, m, code, "cuda")
        ws_grad = torch.empty(ldk.lib().ldk_kernel_grad_workspace_bytes(1, d, 0, n, 0),
                              dtype=torch.uint8, device="cuda")
        reps = []
        for r in range(R):
            ps_r = ldk.PointSet("dnet", 1, d, m, ps.gen[r:r + 1], None, ps.shift[r:r + 1],
                                per_replication=True)
            reps.append((ps_r, *(b[k][r:r + 1] for k in ("k1", "lam", "y", "g", "a", "kg", "L",
                                                           "ds"))))

        def step():
            for ps_r, k1, lam, y, g, a, kg, L, ds in reps:
                ldk.kernel_column(kern, ps_r, 0, n, dtype=dt, out=k1)
                ldk.eig("dnet", k1, out=lam, ws=ws_eig)
                ldk._check(ldk.lib().ldk_mll(ldk.DNET_B2, 1, m, code, ldk._ptr(lam), w["sigma2"],
                                             ldk._ptr(y), ldk._ptr(L), ldk._ptr(g), ldk._ptr(ds),
                                             ldk._ptr(ws_mll), ldk._stream()), "ldk_mll")
                ldk.mll_adjoint("dnet", g, out=a)
                ldk.kernel_grad(kern, ps_r, 0, n, a, dtype=dt, out=kg, ws=ws_grad, k1=k1)

        step()
        torch.cuda.synchronize()
        ms = time_graph(step, K)
        grad = torch.cat([b["kg"], b["ds"][:, None]], dim=1).cpu().numpy()
        return dict(ms=ms, grad=grad)

    r32 = run(torch.float32)
    r32_b = with_engine(0, lambda: run(torch.float32, per_op=False))
    r32_m = with_engine(1, lambda: run(torch.float32, per_op=False))
    r64 = run(torch.float64)
    p32 = run_plain(torch.float32)

    def gerr(r):
        return float(np.max(np.abs(r["grad"] - r64["grad"])) / np.max(np.abs(r64["grad"])))

    err = gerr(r32)
    # factor evaluations of the gradient kernel: one sweep, the forward
    # column supplies the product of the factors
    evals = R * n * d
    kg_ms = r32["per_op"]["kernel_grad"]
    return {
        "workload": "net_m16_d64_r64_dsi2_grad (64 replications of an LMS+DS base-2 net, "
                    "n=2^16, d=64, order-2 DSI kernel, gamma_j=1/j^2, sigma^2=1e-3): "
                    "kernel_column + eig + mll + mll_adjoint + kernel_grad per step",
        "value": round(R / (r32["ms"] * 1e-3), 1),
        "unit": "replication gradients/s",
        "ms_per_step": round(r32["ms"], 5),
        "ms_per_step_f64": round(r64["ms"], 5),
        "ops_ms": {nm: round(r32["per_op"][nm], 5) for nm in names},
        "ops_ms_f64": {nm: round(r64["per_op"][nm], 5) for nm in names},
        "kernel_grad_factor_evals_per_s": round(evals / (kg_ms * 1e-3), 1),
        "f32_grad_rel_err_vs_f64": err,
        "f32_transform_of_y": {
            "butterflies": {"ms_per_step": round(r32_b["ms"], 5),
                            "grad_rel_err_vs_f64": gerr(r32_b)},
            "split16": {"ms_per_step": round(r32_m["ms"], 5), "grad_rel_err_vs_f64": gerr(r32_m)}},
        "plain_per_replication": {"ms_per_step": round(p32["ms"], 5),
                                  "value": round(R / (p32["ms"] * 1e-3), 1),
                                  "grad_rel_err_vs_f64": gerr(p32),
                                  "note": "FP32, the same five calls for one replication at a "
                                          "time (64 x 5 launches per step)"},
        "speedup_vs_plain": round(p32["ms"] / r32["ms"], 2),
        "dtype": "f32 kernel factors and transform of y; f64 eigenvalues, g, adjoint, sums",
    }


def higher_order_bench(K):
    """Order-2 higher-order LMS + digitally shifted net (Sec. 4.3, digital
    interlacing): 64 source dimensions interlaced pairwise into d = 32,
    n = 2^20, one replication.  Times the interlacing of the scrambled
    columns, the point words (HBM roofline) and the order-2 DSI first column
    on the interlaced net (points regenerated)."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    alpha, d, m = 2, 32, 20
    n = 2**m
    src = W.small_net(2502, m=m, d=alpha * d, R=1)

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps = ldk.PointSet("dnet", 1, alpha * d, m, dev_u64(src["gen"]), dev_u64(src["lms"]), None)
    shift = dev_u64(np.random.default_rng(2503).integers(0, 2**62, size=(1, d), dtype=np.uint64))
    cols = torch.empty((1, d, m), dtype=torch.int64, device="cuda")
    hp = ldk.interlace(ps, alpha, shift=shift, out=cols)
    kern = ldk.Kernel("dnet", np.full(d, alpha, np.int32),
                      torch.from_numpy(1.0 / np.arange(1, d + 1, dtype=np.float64) ** 2).cuda(), 1.0)
    pts = torch.empty((1, n, d), dtype=torch.int64, device="cuda")
    k1 = torch.empty((1, n), dtype=torch.float64, device="cuda")
    ms_il = time_graph(lambda: ldk.interlace(ps, alpha, shift=shift, out=cols), K)
    ms_gen = time_graph(lambda: ldk.gen_points(hp, 0, n, out=pts), K)
    ms_kc = time_graph(lambda: ldk.kernel_column(kern, hp, 0, n, out=k1), K)
    gb = 8 * n * d / (ms_gen * 1e-3) / 1e9
    return {"workload": "net_m20_d32_order2_interlaced (LMS on 64 source dimensions, interlaced "
                        "pairwise into d=32, digital shift, n=2^20, order-2 DSI kernel)",
            "interlace_ms": round(ms_il, 5), "gen_points_ms": round(ms_gen, 5),
            "gen_points_GB_s": round(gb, 1), "gen_points_hbm_frac": round(gb / HBM_PEAK_GBS, 4),
            "kernel_column_ms": round(ms_kc, 5),
            "kernel_column_factor_evals_per_s": round(n * d / (ms_kc * 1e-3), 1)}


def cubature_bench(K, lam, y, w):
    """Kernel cubature on the step's eigenvalues (lattice, n = 2^20, d = 32):
    the Bayesian-cubature posterior of the integral from the responses, and
    the squared worst-case errors of 16 weight vectors (Sec. kernel
    computations).  Algorithmic bytes: each transformed row (8 n) and its
    eigenvalue row (8 n) read once."""
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    R, n = y.shape
    m = n.bit_length() - 1
    nw = 16
    om = torch.from_numpy(W.cubature_weights(2504, R, nw, n)).cuda()
    e2 = torch.empty((R, nw), dtype=torch.float64, device="cuda")
    bc = torch.empty((R, len(ldk.BC_FIELDS)), dtype=torch.float64, device="cuda")
    ws_w = ldk._workspace(ldk.OP_WCE, ldk.LATTICE, R * nw, m, ldk.F64, "cuda")
    ws_b = ldk._workspace(ldk.OP_BAYES_CUBATURE, ldk.LATTICE, R, m, ldk.F64, "cuda")
    ms_bc = time_graph(lambda: ldk.bayes_cubature("lattice", lam, w["sigma2"], w["zeta"], y,
                                                  out=bc, ws=ws_b), K)
    ms_w = time_graph(lambda: ldk.wce("lattice", lam, om, w["zeta"], out=e2, ws=ws_w), K)
    f = bc[0].cpu().tolist()
    return {"workload": "lattice_m20_d32_si2 eigenvalues, responses of the step; 16 weight "
                        "vectors around 1/n",
            "bayes_cubature_ms": round(ms_bc, 5),
            "bayes_cubature_GB_s": round(16 * n * R / (ms_bc * 1e-3) / 1e9, 1),
            "wce_ms": round(ms_w, 5), "wce_rules_per_s": round(R * nw / (ms_w * 1e-3), 1),
            "wce_GB_s": round(16 * n * R * nw / (ms_w * 1e-3) / 1e9, 1),
            "posterior": {k: f[i] for i, k in enumerate(ldk.BC_FIELDS)},
            "wce2_equal_weights": float(e2[0, 0].cpu())}


def rqmc_bench(K, probe=False):
    """RQMC estimate + Student-t interval of the corner-peak integrand
    (eq. RQMC), points regenerated in the kernel: the paper's example shape
    (d = 50, n = 2^15, R = 10, order-3 interlaced LMS + shifted net) and a
    throughput shape (d = 50, n = 2^20, R = 16; shifted lattice and LMS net).
    Cost unit: point coordinates (n d R per estimate).  probe: K eager calls
    of each, no graphs and no timing (for counter runs)."""
    import ctypes as C

    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    d = 50
    coef = torch.from_numpy(W.corner_peak_coefficients(d)).cuda()
    res = {}

    def timed(name, ps, n):
        mu_r = torch.empty(ps.R, dtype=torch.float64, device="cuda")
        st = torch.empty(3, dtype=torch.float64, device="cuda")
        ws = torch.empty(max(int(ldk.lib().ldk_rqmc_workspace_bytes(C.byref(ps._c()), n)), 1),
                         dtype=torch.uint8, device="cuda")
        def call():
            ldk.rqmc(ps, n, "corner_peak", coef, mu_r=mu_r, stats=st, ws=ws)

        if probe:
            for _ in range(K):
                call()
            return
        ms = time_graph(call, K)
        v = st.cpu().tolist()
        res[name] = {"ms": round(ms, 5), "coords_per_s": round(n * d * ps.R / (ms * 1e-3), 1),
                     "mean": v[0], "half_width_99": v[2]}

    m, R, alpha = 15, 10, 3
    src = W.small_net(2502, m=m, d=alpha * d, R=R)
    shift = np.random.default_rng(7).integers(0, 2**64, size=(R, d), dtype=np.uint64)
    ps_src = ldk.PointSet("dnet", R, alpha * d, m, dev_u64(src["gen"]), dev_u64(src["lms"]), None)
    hp = ldk.interlace(ps_src, alpha, shift=dev_u64(shift))
    timed("paper_shape_net_order3_m15_d50_R10", hp, 2**m)
    m, R = 20, 16
    wl = W.small_lattice(2506, m, d, R)
    timed("lattice_m20_d50_R16", ldk.PointSet("lattice", R, d, m, dev_u64(wl["gen"]), None,
                                              dev_u64(wl["shift"])), 2**m)
    wn = W.small_net(2507, m, d, R)
    timed("net_lms_m20_d50_R16", ldk.PointSet("dnet", R, d, m, dev_u64(wn["gen"]),
                                              dev_u64(wn["lms"]), dev_u64(wn["shift"])), 2**m)
    return res


def structure_free_bench(K):
    """The point sets without fast-transform structure (they feed QMC means):
    Halton and Faure (b = 53) with LMS and digit permutations, and a base-2
    net under nested uniform scrambling, d = 52 and R = 16 as in the paper's
    listings, at n = 2^16: coordinate generation and the RQMC corner-peak
    estimate over the generated points, device time per launch (graph
    replays)."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    R, d, m = 16, 52, 16
    n = 2**m
    coef = torch.from_numpy(W.corner_peak_coefficients(d)).cuda()
    out = {}
    for name, kind, base in (("halton_lms_dp", "halton", 0), ("faure53_lms_dp", "faure", 53),
                             ("net_nus", "nus", 0)):
        if kind == "nus":
            t = W.small_net(31, m, d, 1)
            ps = ldk.BPointSet("nus", R, d, m=m,
                               gen=torch.from_numpy(t["gen"].view(np.int64).copy()).cuda(),
                               seed=torch.from_numpy(W.nus_seeds(31, R, d).view(np.int64)).cuda())
        else:
            inp = W.bpoint_inputs(31, kind, R, d, base=base)
            ps = ldk.BPointSet(kind, R, d, base=base, flags=ldk.BR_LMS | ldk.BR_DP,
                               **{k: torch.from_numpy(v).cuda() for k, v in inp.items()})
        x = torch.empty((R, n, d), dtype=torch.float64, device="cuda")
        ws = torch.empty(max(ldk.lib().ldk_bpoints_workspace_bytes(C_ref(ps)), 256),
                         dtype=torch.uint8, device="cuda")
        ms_gen = time_graph(lambda: ldk.gen_bpoints(ps, 0, n, out=x, ws=ws), K)
        mu_r = torch.empty(R, dtype=torch.float64, device="cuda")
        st = torch.empty(3, dtype=torch.float64, device="cuda")
        wsr = torch.empty(ldk.lib().ldk_rqmc_points_workspace_bytes(R, n), dtype=torch.uint8,
                          device="cuda")
        ms_rq = time_graph(lambda: ldk.rqmc_points(x, "corner_peak", coef, mu_r=mu_r, stats=st,
                                                   ws=wsr), K)
        stats = st.cpu().numpy()
        out[name] = {"gen_ms": round(ms_gen, 5), "coords_per_s": round(R * n * d / (ms_gen * 1e-3), 1),
                     "gen_GB_s": round(8 * R * n * d / (ms_gen * 1e-3) / 1e9, 1),
                     "rqmc_ms": round(ms_rq, 5),
                     "rqmc_GB_s": round(8 * R * n * d / (ms_rq * 1e-3) / 1e9, 1),
                     "mean": float(stats[0]), "half_width_99": float(stats[2])}
        del x
    out["workload"] = (f"R={R} randomizations, d={d}, n=2^{m} points each; corner-peak "
                       "integrand of the RQMC example over the generated coordinates")
    return out


def structure_free_probe():
    """The structure-free generators and the RQMC estimate over their
    coordinates (the shapes of structure_free_bench), three eager calls each
    and no graphs, for counter runs."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    R, d, m = 16, 52, 16
    n = 2**m
    coef = torch.from_numpy(W.corner_peak_coefficients(d)).cuda()
    x = torch.empty((R, n, d), dtype=torch.float64, device="cuda")
    for kind, base in (("halton", 0), ("faure", 53), ("nus", 0)):
        if kind == "nus":
            t = W.small_net(31, m, d, 1)
            ps = ldk.BPointSet("nus", R, d, m=m,
                               gen=torch.from_numpy(t["gen"].view(np.int64).copy()).cuda(),
                               seed=torch.from_numpy(W.nus_seeds(31, R, d).view(np.int64)).cuda())
        else:
            inp = W.bpoint_inputs(31, kind, R, d, base=base)
            ps = ldk.BPointSet(kind, R, d, base=base, flags=ldk.BR_LMS | ldk.BR_DP,
                               **{k: torch.from_numpy(v).cuda() for k, v in inp.items()})
        ws = torch.empty(max(ldk.lib().ldk_bpoints_workspace_bytes(C_ref(ps)), 256),
                         dtype=torch.uint8, device="cuda")
        for _ in range(3):
            ldk.gen_bpoints(ps, 0, n, out=x, ws=ws)
            ldk.rqmc_points(x, "corner_peak", coef)
    torch.cuda.synchronize()


def C_ref(ps):
    import ctypes as C

    return C.byref(ps._c())


def update_bench(K):
    """Doubling n from 2^19 to 2^20 on the net workload (workload 3: LMS +
    digitally shifted net, d = 32, order-4 DSI kernel, FP64), against fresh
    work at 2^20: (a) the transformed responses, update_double against a
    fresh FWHT; (b) extending a fit's inputs, i.e. the point words and first
    column of the new half, the eigenvalue update and the ỹ update, against
    points + column, eigenvalues and the transform of all 2^20 points."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    w = W.workload(3)
    m, d, R = w["m"], w["d"], w["R"]
    n, h = 2**m, 2 ** (m - 1)

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps = ldk.PointSet("dnet", R, d, m, dev_u64(w["gen"]), dev_u64(w["lms"]), dev_u64(w["shift"]))
    kern = ldk.Kernel("dnet", w["alpha"], torch.from_numpy(np.asarray(w["gamma"], np.float64)).cuda(),
                      w["zeta"])
    y = torch.from_numpy(np.ascontiguousarray(w["y"][:, 0, :])).cuda()
    pts_full = torch.empty((R, n, d), dtype=torch.int64, device="cuda")
    k1_full = torch.empty((R, n), dtype=torch.float64, device="cuda")
    pts_new = torch.empty((R, h, d), dtype=torch.int64, device="cuda")
    k1_new = torch.empty((R, h), dtype=torch.float64, device="cuda")
    ldk.points_column(kern, ps, 0, n, pts=pts_full, k1=k1_full)
    lam_old = ldk.eig("dnet", k1_full[:, :h].contiguous())
    yt_old = ldk.transform("dnet", y[:, :h].contiguous())
    y_new = y[:, h:].contiguous()
    yt = torch.empty((R, n), dtype=torch.float64, device="cuda")
    lam = torch.empty((R, n), dtype=torch.float64, device="cuda")
    ms_upd = time_graph(lambda: ldk.update_double("dnet", yt_old, y_new, out=yt), K)
    ms_fresh = time_graph(lambda: ldk.transform("dnet", y, out=yt), K)

    def extend():
        ldk.points_column(kern, ps, h, n, pts=pts_new, k1=k1_new)
        ldk.eig_update_double("dnet", lam_old, k1_new, out=lam)
        ldk.update_double("dnet", yt_old, y_new, out=yt)

    def fresh():
        ldk.points_column(kern, ps, 0, n, pts=pts_full, k1=k1_full)
        ldk.eig("dnet", k1_full, out=lam)
        ldk.transform("dnet", y, out=yt)

    ms_ext = time_graph(extend, K)
    ms_fit = time_graph(fresh, K)
    alg = 16 * n * R  # read the old half's transform and the new half, write 2^20 (FP64)
    return {"workload": "net_m20_d32_dsi4 (LMS + digital shift, n = 2^19 -> 2^20, FP64)",
            "update_double_ms": round(ms_upd, 5), "fresh_transform_ms": round(ms_fresh, 5),
            "update_double_GB_s": round(alg / (ms_upd * 1e-3) / 1e9, 1),
            "extend_ms": round(ms_ext, 5), "fresh_ms": round(ms_fit, 5),
            "extend_speedup": round(ms_fit / ms_ext, 3)}


def fwht_bench(K):
    """The net workload's transform at n = 2^20: one FP32 row of responses,
    and 16 rows (the workload's response with 15 seeded normal rows): FP32
    butterfly passes against the split-FP16 matrix-core passes, device time
    per launch (graph replays) and each one's normwise error against the
    FP64 transform of the same rows."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    w = W.workload(3)
    row = np.ascontiguousarray(w["y"][:, 0, :])
    extra = np.random.default_rng(20260).standard_normal((15, row.shape[1]))
    res = {}
    for B in (1, 16):
        x64 = torch.from_numpy(np.concatenate([row, extra[:B - 1]])).cuda()
        x32 = x64.float()
        ref = ldk.transform("dnet", x64)
        y_b, y_m = torch.empty_like(x32), torch.empty_like(x32)
        ms_b = time_graph(lambda: ldk.transform("dnet", x32, out=y_b), K)
        ms_m = time_graph(lambda: ldk.fwht_split16(x32, out=y_m), K)

        def err(y):
            return float(torch.linalg.norm(y.double() - ref) / torch.linalg.norm(ref))

        nbytes = 2 * 4 * x32.numel()
        res[f"rows{B}"] = {
            "n": x32.shape[1], "rows": B, "fp32_butterflies_ms": round(ms_b, 5),
            "split16_mfma_ms": round(ms_m, 5),
            "fp32_butterflies_GB_s": round(nbytes / (ms_b * 1e-3) / 1e9, 1),
            "split16_mfma_GB_s": round(nbytes / (ms_m * 1e-3) / 1e9, 1),
            "split16_over_butterflies": round(ms_m / ms_b, 3),
            "fp32_butterflies_rel_err": err(y_b), "split16_mfma_rel_err": err(y_m)}
        del x64, x32, y_b, y_m, ref
    res["bytes"] = "read + write of the FP32 rows once (each engine makes two passes at 2^20)"
    return res


def batch_bench(K, warmup):
    """Instance table of 256 problems of mixed kind (rank-1 lattice with SI
    order 2, or LMS+DS net with DSI order 2) and size n = 2^12 .. 2^18, d = 16,
    8 right-hand sides each, FP64: first column, eigenvalues, 8 solves and the
    log-det per instance.  Batched: the library's batch plan (instances of
    one (kind, m) run as the replications of one point set, one first-column
    launch and one fit per group, groups over 1 or 4 streams), captured once
    as a HIP graph.  Plain: the same calls instance by instance (one launch
    per op per instance), also captured as one graph.  Graphs are replayed K
    times between HIP events."""
    import numpy as np
    import torch

    from paper_2502_14256_amd.batch import BatchFit, Instance
    import workloads as W

    w = W.workload(4)
    inst = [Instance(kind=t["kind"], m=t["m"], shift=t["shift"][0],
                     lms=None if t["lms"] is None else t["lms"][0], y=t["y"][0])
            for t in w["instances"]]
    main = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record(main)
        for _ in range(K):
            fn()
        e.record(main)
        torch.cuda.synchronize()
        return a.elapsed_time(e) / K

    res = {}
    for streams in (1, 4):
        b = BatchFit(inst, {"lattice": w["lattice_gen"], "dnet": w["net_gen"]}, w["m_max"],
                     w["alpha"], w["gamma"], w["zeta"], w["sigma2"], streams=streams)
        b.capture()
        torch.cuda.synchronize()
        res[streams] = (timed(b.step), b.kernel_nodes(), b.n_groups)
        if streams == 1:
            # the plain reference: every instance with the separate entry points
            g = torch.cuda.CUDAGraph()
            b.step_plain()
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                b.step_plain()
            ms_p = timed(g.replay)
        del b
    best = min(res, key=lambda k: res[k][0])
    ms_b = res[best][0]
    ns = np.array([2 ** t["m"] for t in w["instances"]], dtype=np.int64)
    solves = len(ns) * w["nrhs"]
    alg = int((2 * 8 * w["nrhs"] + 8) * ns.sum())  # read y, write c, read lambda (FP64)

    # FP32: first column, responses, solutions and solve transforms in FP32
    # (eigenvalues, division and log-det in FP64); net solves on the FP32
    # butterflies or the split-FP16 matrix cores; per-instance errors
    # against the FP64 batched results (themselves held to the FP64 oracle
    # by the parity tests)
    gens = {"lattice": w["lattice_gen"], "dnet": w["net_gen"]}
    b64 = BatchFit(inst, gens, w["m_max"], w["alpha"], w["gamma"], w["zeta"], w["sigma2"],
                   streams=best)
    b64.step()
    torch.cuda.synchronize()
    c64 = [b64.c(i).cpu().numpy() for i in range(len(inst))]
    ld64 = np.array([b64.logdet(i).item() for i in range(len(inst))])
    del b64

    def f32_leg(plain):
        b = BatchFit(inst, gens, w["m_max"], w["alpha"], w["gamma"], w["zeta"], w["sigma2"],
                     dtype=torch.float32, streams=best)
        if plain:
            g = torch.cuda.CUDAGraph()
            b.step_plain()
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                b.step_plain()
            ms = timed(g.replay)
        else:
            b.capture()
            torch.cuda.synchronize()
            ms = timed(b.step)
        ec = np.array([np.linalg.norm(b.c(i).double().cpu().numpy() - c64[i])
                       / np.linalg.norm(c64[i]) for i in range(len(inst))])
        eld = np.array([abs(b.logdet(i).item() - ld64[i]) / abs(ld64[i])
                        for i in range(len(inst))])
        del b
        return {"ms_per_step": round(ms, 4), "solves_per_s": round(solves / (ms * 1e-3), 1),
                "err_c_vs_f64_max": float(ec.max()), "err_c_vs_f64_median": float(np.median(ec)),
                "err_c_vs_f64_net_max": float(max(e for e, t in zip(ec, w["instances"])
                                                  if t["kind"] == "dnet")),
                "err_logdet_vs_f64_max": float(eld.max())}

    f32 = {"batched_split16": with_engine(1, lambda: f32_leg(False)),
           "batched_butterflies": with_engine(0, lambda: f32_leg(False)),
           "plain_butterflies": with_engine(0, lambda: f32_leg(True))}
    return {
        "workload": "batched_256_mixed_d16 (256 instances, kind lattice/net at random, "
                    "n=2^12..2^18, d=16, 8 RHS, FP64): kernel_column + eig + solve + logdet "
                    "per instance",
        "value": round(solves / (ms_b * 1e-3), 1),
        "unit": "solves/s",
        "ms_per_step": round(ms_b, 4),
        "streams": best,
        "ms_per_step_by_streams": {str(k): round(v[0], 4) for k, v in res.items()},
        "kernel_launches_per_step": res[best][1],
        "groups": res[best][2],
        "plain_solves_per_s": round(solves / (ms_p * 1e-3), 1),
        "plain_ms_per_step": round(ms_p, 4),
        "plain_launches_per_step": 4 * len(ns),
        "speedup_vs_plain": round(ms_p / ms_b, 2),
        "solve_alg_bytes": alg,
        "solve_equivalent_GB_s": round(alg / (ms_b * 1e-3) / 1e9, 1),
        "solve_equivalent_hbm_frac": round(alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "f32": f32,
        "f32_note": "FP32 column, responses, solutions and solve transforms; FP64 eigenvalues, "
                    "division and log-det; errors per instance against the FP64 batched "
                    "results (normwise c; relative log-det)",
    }


def solve_rhs_bench(K, lam_lat, w_lat):
    """Gram solves with cached eigenvalues at n = 2^20 in FP64 and FP32
    (responses, solution and transforms; lambda FP64), one and 16
    right-hand sides, on the lattice workload's eigenvalues and on the net
    workload's (n = 2^20, d = 32, order-4 DSI kernel): solves per second and
    the fraction of the 8 TB/s HBM peak, with algorithmic bytes 2 s n per
    right-hand side (read y, write c) plus 8 n for lambda, read once."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    w3 = W.workload(3)
    n = 2 ** w3["m"]

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps3 = ldk.PointSet("dnet", 1, w3["d"], w3["m"], dev_u64(w3["gen"]), dev_u64(w3["lms"]),
                       dev_u64(w3["shift"]))
    k3 = ldk.Kernel("dnet", w3["alpha"],
                    torch.tensor(w3["gamma"], dtype=torch.float64, device="cuda"), w3["zeta"])
    lam_net = ldk.eig("dnet", ldk.kernel_column(k3, ps3, 0, n))
    rng = np.random.default_rng(99)
    res = {}
    for kind, lam, s2 in (("lattice", lam_lat, w_lat["sigma2"]), ("net", lam_net, w3["sigma2"])):
        kd = "lattice" if kind == "lattice" else "dnet"
        for dt, sfx in ((torch.float64, ""), (torch.float32, "_f32")):
            row = {}
            esz = 8 if dt == torch.float64 else 4
            for nrhs in (1, 16):
                y = torch.from_numpy(rng.standard_normal((1, nrhs, n))).cuda().to(dt)
                c = torch.empty_like(y)
                ws = ldk._workspace(ldk.OP_SOLVE, ldk._kind(kd), nrhs, w3["m"], ldk._dtype_code(dt),
                                    "cuda")
                ms = time_graph(lambda: ldk.solve(kd, lam, s2, y, out=c, ws=ws), K)
                alg = (2 * esz * nrhs + 8) * n
                gbs = alg / (ms * 1e-3) / 1e9
                row[f"rhs{nrhs}"] = {"ms": round(ms, 5), "solves_per_s": round(nrhs / (ms * 1e-3), 1),
                                     "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
                del y, c, ws
            res[kind + sfx] = row
    res["bytes"] = ("algorithmic: 2 s n per right-hand side (read y, write c; s = 8 FP64, 4 FP32) "
                    "+ 8 n (lambda, FP64, read once)")
    return res


def fp32_step_bench(K, kern, ps, w, y_host, c64):
    """The same step in FP32: the first column, the responses, the solution
    and the solve transforms in FP32 (the eigenvalues, the division by
    lambda + sigma^2 and the log-det stay FP64): time per step and the
    solution's normwise difference from the FP64 step's."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk

    n, R = 2 ** w["m"], w["R"]
    y = torch.from_numpy(y_host).to(device="cuda", dtype=torch.float32)
    pts = torch.empty((R, n, w["d"]), dtype=torch.int64, device="cuda")
    k1 = torch.empty((R, n), dtype=torch.float32, device="cuda")
    lam = torch.empty((R, n), dtype=torch.float64, device="cuda")
    c = torch.empty_like(y)
    ld = torch.empty(R, dtype=torch.float64, device="cuda")
    ws = ldk._workspace(ldk.OP_FIT, ldk.LATTICE, 2 * R, w["m"], ldk.F32, "cuda")

    def step():
        ldk.points_column(kern, ps, 0, n, dtype=torch.float32, pts=pts, k1=k1)
        ldk.fit("lattice", k1, w["sigma2"], y, lam=lam, c=c, logdet=ld, ws=ws)

    ms = time_graph(step, K)
    ch = c.double().cpu().numpy()
    c64h = c64.double().cpu().numpy()
    return {"ms_per_step": round(ms, 5), "solves_per_s": round(R / (ms * 1e-3), 2),
            "rel_c_vs_fp64_gpu_step": float(np.linalg.norm(ch - c64h) / np.linalg.norm(c64h)),
            "dtype": "f32 first column, responses, solution and solve transforms; f64 "
                     "eigenvalues, division and log-det", "_c": ch}


def c1_latency_bench(K):
    """The plain small problem (net n = 1024, d = 4, order-1 DSI kernel,
    sigma^2 = 1e-8): points, first column, eigenvalues, solve and log-det,
    as one captured graph (device time per replay, median and minimum over
    five runs of K replays) and issued eagerly from the host (wall time per
    call, synchronised)."""
    import numpy as np
    import torch

    import paper_2502_14256_amd as ldk
    import workloads as W

    w = W.workload(1)
    n = 2 ** w["m"]

    def dev_u64(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64).copy()).cuda()

    ps = ldk.PointSet("dnet", 1, w["d"], w["m"], dev_u64(w["gen"]), dev_u64(w["lms"]),
                      dev_u64(w["shift"]))
    kern = ldk.Kernel("dnet", w["alpha"],
                      torch.tensor(w["gamma"], dtype=torch.float64, device="cuda"), w["zeta"])
    y = torch.from_numpy(np.ascontiguousarray(w["y"])).cuda()
    pts = torch.empty((1, n, w["d"]), dtype=torch.int64, device="cuda")
    k1 = torch.empty((1, n), dtype=torch.float64, device="cuda")
    lam = torch.empty((1, n), dtype=torch.float64, device="cuda")
    c = torch.empty_like(y)
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = ldk._workspace(ldk.OP_FIT, ldk.DNET_B2, 2, w["m"], ldk.F64, "cuda")

    def step():
        ldk.points_column(kern, ps, 0, n, pts=pts, k1=k1)
        ldk.fit("dnet", k1, w["sigma2"], y, lam=lam, c=c, logdet=ld, ws=ws)

    # a replay takes about 20 us, so single runs of K replays scatter:
    # the median of five runs is the figure
    st = time_graph_stats(step, K)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
        torch.cuda.synchronize()
    eager_us = (time.perf_counter() - t0) / K * 1e6
    return {"workload": "net_m10_d4_dsi1 (LMS + shift, n=1024, d=4, order-1 DSI, "
                        "sigma^2=1e-8)", "graph_us": round(st["median"] * 1e3, 2),
            "graph_us_min": round(st["min"] * 1e3, 2), "graph_runs": st["runs"],
            "eager_synchronised_us": round(eager_us, 1)}


def cpu_baseline(w, y):
    """The oracle (plain C, FP64) timed on this host on the same whole step
    (points, first column, FFTBR eigenvalues, solve, log-det at n = 2^20,
    d = 32).  Built here with -O3 -march=native -ffp-contract=off -fopenmp
    (bit for bit the results of the test build; the OpenMP pragmas share out
    points, kernel-column entries and each transform stage's butterflies).
    Two legs: one thread, and every thread the host offers this process
    (OMP_NUM_THREADS when set, else the CPU count); each the median of 5
    steps after 1 warm-up.  The responses y are synthesised outside the timed
    steps.  Returns (record, the oracle's solution c)."""
    import statistics
    import tempfile

    import numpy as np

    import oracle

    tmp = tempfile.mkdtemp(prefix="orc_baseline_")
    so = oracle.build(path=os.path.join(tmp, "liborc_baseline.so"),
                      flags=("-O3", "-march=native", "-ffp-contract=off", "-fopenmp"))
    oracle.use_library(so)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count()
    all_threads = int(os.environ.get("OMP_NUM_THREADS") or nproc)
    c_out = None

    def step():
        nonlocal c_out
        pts = oracle.points(w)
        k1 = oracle.kernel_column("lattice", pts, pts[:, 0], w["alpha"], w["gamma"], w["zeta"])
        lam, _ = oracle.eig("lattice", k1)
        c_out = oracle.solve("lattice", lam, w["sigma2"], y)
        oracle.logdet(lam, w["sigma2"])

    legs = {}
    for name, threads in (("single", 1), ("all", all_threads)):
        oracle.lib().orc_set_threads(threads)
        used = oracle.lib().orc_threads()
        step()  # warm-up
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            step()
            times.append(time.perf_counter() - t0)
        legs[name] = {"threads": used, "median_s": round(statistics.median(times), 4),
                      "solves_per_s": round(1.0 / statistics.median(times), 5)}
    oracle.use_library(None)
    rec = {"value": legs["all"]["solves_per_s"], "unit": "solves/s",
           "cores": legs["all"]["threads"], "kind": "oracle",
           "sample": "median of 5 whole steps after 1 warm-up (points, first column, FFTBR "
                     "eigenvalues, solve, log-det at n=2^20, d=32, FP64), C oracle built on "
                     "this host with -O3 -march=native -ffp-contract=off -fopenmp",
           "single_thread": legs["single"], "all_threads": legs["all"],
           "nproc": nproc, "cpu_model": model}
    return rec, c_out[:, 0, :] if c_out.ndim == 3 else c_out


if __name__ == "__main__":
    main()
