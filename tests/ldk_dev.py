"""Helpers for GPU tests: move workload arrays to the device and back, and the
tolerance arithmetic used by the parity tests.  No arithmetic of the method."""
import math

import numpy as np
import torch

import paper_2502_14256_amd as ldk

U64_EPS = 2.0**-53
F32_EPS = 2.0**-24


def dev_u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64).copy()).cuda()


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def pointset(w, order=None):
    return ldk.PointSet(
        kind=w["kind"], R=w["R"], d=w["d"], m_max=w.get("m_max", w["m"]),
        gen=dev_u64(w["gen"]),
        lms=None if w.get("lms") is None else dev_u64(w["lms"]),
        shift=None if w.get("shift") is None else dev_u64(w["shift"]),
        order=order or w.get("order", "natural"))


def kernel(w):
    return ldk.Kernel(kind=w["kind"], alpha=np.asarray(w["alpha"], np.int32),
                      gamma=torch.as_tensor(np.asarray(w["gamma"], np.float64)).cuda(),
                      zeta=float(w["zeta"]))


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def kernel_scale(w):
    """zeta prod_j (1 + gamma_j max|K_alpha_j|): bound on |k1| used to scale the
    elementwise absolute tolerance of the first column (a factor 1 + gamma K
    can cross zero, so a purely relative test is ill-posed)."""
    import math
    if w["kind"] == "lattice":
        kmax = {1: math.pi**2 / 3, 2: math.pi**4 / 45, 3: 2 * math.pi**6 / 945}
    else:
        kmax = {1: 2.0, 2: 1.5, 3: 2.0, 4: 2.5}
    s = float(w["zeta"])
    for a, g in zip(np.asarray(w["alpha"]), np.asarray(w["gamma"])):
        s *= 1.0 + abs(g) * kmax[int(a)]
    return s


def solve_tol(lam, sigma2, y, c, m, eps):
    """Normwise first-order bound on the relative error of
    c = V diag(1/(lambda + s2)) conj(V) y computed with two transforms of
    log2(n) butterfly stages and one division each rounded at eps:
    |dc| <= (2 m + 2) eps ||D|| ||y||, D = diag(1/(lambda + s2)), divided by
    ||c||, with a factor 4 of headroom."""
    lam = np.asarray(lam, np.float64)
    y = np.asarray(y, np.float64)
    c = np.asarray(c, np.float64)
    dmax = 1.0 / np.min(lam + sigma2, axis=-1)
    R = lam.shape[0]
    ratio = max(dmax[r] * np.linalg.norm(y[r]) / max(np.linalg.norm(c[r]), 1e-300)
                for r in range(R))
    return 4.0 * (2 * m + 2) * eps * ratio


def record(name, **vals):
    """Append measured errors as one JSON line to the file named by the
    environment variable LDK_ERROR_LOG (nothing when it is unset)."""
    import json
    import os
    path = os.environ.get("LDK_ERROR_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **{k: float(v) for k, v in vals.items()}}) + "\n")



def gate_vs_ld(got, ref, ref_ld, eps, floor):
    """Conditioning-aware gate of a GPU result against the FP64 oracle: the
    FP64 oracle's own error e_dd = |ref - ref_ld| (ref_ld: its long-double
    twin on the same input) measures how this input amplifies rounding; a
    GPU result computed in arithmetic of unit roundoff eps may be off by
    10 e_dd (eps / 2^-53) (10x headroom, error linear in the unit roundoff of
    the steps run at eps), and never needs to be better than floor * |ref|
    (the stated tolerance).  FP32 steps also keep only the top 32 digits of
    each coordinate before rounding them to 24 bits, an absolute 2^-32 on
    top of the relative 2^-24 that has no FP64 counterpart; it doubles the
    coordinate error for x >= 2^-8, hence a factor 2 for eps > 2^-53.
    Normwise over the last axis; returns (error / gate) per row."""
    got, ref, ref_ld = (np.atleast_2d(np.asarray(a, np.float64)) for a in (got, ref, ref_ld))
    e_dd = np.max(np.abs(ref - ref_ld), axis=-1)
    scale = np.max(np.abs(ref_ld), axis=-1)
    coord = 2.0 if eps > U64_EPS else 1.0
    gate = np.maximum(10.0 * coord * e_dd * (eps / U64_EPS), floor * scale)
    return np.max(np.abs(got - ref), axis=-1) / gate
