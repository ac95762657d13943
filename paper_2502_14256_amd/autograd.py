"""Gaussian-process marginal log-likelihood with gradients in the kernel
parameters, as a ``torch.autograd.Function`` over the library's kernels.

The paper motivates fitting the kernel's parameters (Sec. 3) and gives the
eigen-decomposition that makes the likelihood cheap (Sec. 5.4), but prints no
objective; the standard GP one is used, in the eigenbasis (see ldk_mll):

    L_r = -1/2 sum_k |yt_rk|^2 / (lambda_rk + s2) - 1/2 sum_k log(lambda_rk + s2)
          - (n/2) log 2 pi,

one value per replication r (independent data sets sharing the parameters),
with parameters theta = (log gamma_1..d, log zeta, log s2).

Forward: ldk_kernel_column -> ldk_eig -> ldk_mll.  Backward: dL/dlambda from
ldk_mll, its adjoint back to dL/dk1 (ldk_mll_adjoint: the FWHT is
self-adjoint, the lattice map's adjoint is the inverse-direction transform),
then the chain rule through the product kernel (ldk_kernel_grad), and
dL/dlog s2 from ldk_mll.  With ``recompute=True`` (the default) the forward
saves nothing of size n: backward regenerates the points, the first column,
the eigenvalues and dL/dlambda from theta, so the memory held between the
passes is O(d); with ``recompute=False`` forward keeps k1 and dL/dlambda
(two [R][n] arrays) and backward starts from them.  Both give bit-identical
gradients (the same kernels on the same inputs).
"""
from __future__ import annotations

import torch

from . import (Kernel, LdkError, PointSet, _kind, eig, kernel_column, kernel_grad, mll,
               mll_adjoint)


def _kernel(kind: str, alpha, log_gamma: torch.Tensor, log_zeta: torch.Tensor) -> Kernel:
    gamma = torch.exp(log_gamma.detach()).to(torch.float64).contiguous()
    return Kernel(kind, alpha, gamma, float(torch.exp(log_zeta.detach()).item()))


def _forward_parts(ps: PointSet, kind: str, alpha, log_gamma, log_zeta, log_sigma2, y, dtype):
    n = y.shape[-1]
    k = _kernel(kind, alpha, log_gamma, log_zeta)
    k1 = kernel_column(k, ps, 0, n, dtype=dtype)
    lam = eig(kind, k1)
    s2 = float(torch.exp(log_sigma2.detach()).item())
    L, g, ds = mll(kind, lam, s2, y.to(dtype).contiguous())
    return k, k1, L, g, ds


class MarginalLogLikelihood(torch.autograd.Function):
    """L[R] = per-replication GP log marginal likelihood; see the module text.

    apply(log_gamma [d], log_zeta [], log_sigma2 [], ps, kind, alpha, y [R][n],
          dtype, recompute) -> L [R] (float64)."""

    @staticmethod
    def forward(ctx, log_gamma, log_zeta, log_sigma2, ps, kind, alpha, y, dtype, recompute):
        k, k1, L, g, ds = _forward_parts(ps, kind, alpha, log_gamma, log_zeta, log_sigma2, y,
                                         dtype)
        ctx.ps, ctx.kind, ctx.alpha, ctx.dtype, ctx.recompute = ps, kind, alpha, dtype, recompute
        ctx.n = y.shape[-1]
        if recompute:
            ctx.save_for_backward(log_gamma.detach(), log_zeta.detach(), log_sigma2.detach(), y)
        else:
            ctx.save_for_backward(log_gamma.detach(), log_zeta.detach(), log_sigma2.detach(), y,
                                  k1, g, ds)
        return L

    @staticmethod
    def backward(ctx, grad_L):
        saved = ctx.saved_tensors
        log_gamma, log_zeta, log_sigma2, y = saved[:4]
        if ctx.recompute:
            k, k1, _, g, ds = _forward_parts(ctx.ps, ctx.kind, ctx.alpha, log_gamma, log_zeta,
                                             log_sigma2, y, ctx.dtype)
        else:
            k1, g, ds = saved[4:]
            k = _kernel(ctx.kind, ctx.alpha, log_gamma, log_zeta)
        a = mll_adjoint(ctx.kind, g)
        kg = kernel_grad(k, ctx.ps, 0, ctx.n, a, dtype=ctx.dtype, k1=k1)  # [R][d + 1]
        w = grad_L.to(torch.float64).reshape(-1, 1)
        G = torch.cat([kg, ds[:, None]], dim=1) * w  # rows weighted by dL_total / dL_r
        tot = G.sum(dim=0)
        d = kg.shape[1] - 1
        return (tot[:d].to(log_gamma.dtype), tot[d].to(log_zeta.dtype),
                tot[d + 1].to(log_sigma2.dtype), None, None, None, None, None, None)


def marginal_log_likelihood(ps: PointSet, kind, alpha, log_gamma: torch.Tensor,
                            log_zeta: torch.Tensor, log_sigma2: torch.Tensor, y: torch.Tensor,
                            dtype: torch.dtype = torch.float32, recompute: bool = True):
    """Per-replication GP log marginal likelihood L [R] (float64) of responses
    y [R][n] at the points 0 .. n-1 of ps, differentiable in log_gamma [d],
    log_zeta [] and log_sigma2 [] (float64 device tensors).  dtype is the
    precision of the kernel factors and of the transform of y (eigenvalues,
    dL/dlambda, the adjoint and every sum stay FP64)."""
    kd = {0: "lattice", 1: "dnet"}[_kind(kind)]
    if ps.kind not in (kd, _kind(kd)):
        raise LdkError("the point set and the kernel must be of the same kind")
    if y.dim() != 2 or y.shape[0] != ps.R:
        raise LdkError("y must be [R][n]")
    for t, nm in ((log_gamma, "log_gamma"), (log_zeta, "log_zeta"), (log_sigma2, "log_sigma2")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise LdkError(f"{nm} must be a float64 device tensor")
    if log_gamma.numel() != ps.d or log_zeta.numel() != 1 or log_sigma2.numel() != 1:
        raise LdkError("log_gamma must hold d values, log_zeta and log_sigma2 one each")
    return MarginalLogLikelihood.apply(log_gamma, log_zeta.reshape(()), log_sigma2.reshape(()),
                                       ps, kd, alpha, y, dtype, recompute)
