"""Differentiable block solve X = A^-1 B for SPD A (torch.autograd.Function).

Forward: block CG on the device (bkry_cg_solve); the solution X stays on the
device for the backward pass.  Backward, for an upstream gradient G = dL/dX:
    Lambda     = A^-T G        (a second block CG solve; A^T = A for SPD A),
    dL/dB      = Lambda,
    dL/dvalues = -(Lambda X^T) on the pattern of A  (bkry_sddmm, alpha = -1).
Marshalling only: both solves and the sampled product run in the library.

Both gradients are exact only for converged solves: a forward or adjoint
solve that stops at its iteration cap raises SolveNotConverged instead of
returning gradients of an unconverged iterate.
"""
from __future__ import annotations

import torch


class SolveNotConverged(RuntimeError):
    """A solve inside the differentiable block solve missed its tolerance."""


def _require_converged(info, which, opts):
    if not info.get("converged"):
        raise SolveNotConverged(
            f"{which} block CG solve stopped after {info.get('iters')} iterations without reaching "
            f"tol={opts['tol']:g} (maxit={opts['maxit']}); its gradient would be wrong")


class BlockSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, B, A, h, kind="block", q=1, tol=1e-13, maxit=10000, eta=float("inf")):
        from . import CsrMatrix, bkry_cg_solve
        Av = CsrMatrix(A.n, A.rowptr, A.colind, vals.detach().contiguous())
        opts = dict(kind=kind, q=q, tol=tol, maxit=maxit, eta=eta)
        X, info = bkry_cg_solve(h, Av, B.detach().contiguous(), **opts)
        _require_converged(info, "forward", opts)
        ctx.save_for_backward(X)
        ctx.A, ctx.h, ctx.opts = Av, h, opts
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, gX):
        from . import bkry_cg_solve, bkry_sddmm
        (X,) = ctx.saved_tensors
        lam, info = bkry_cg_solve(ctx.h, ctx.A, gX.contiguous(), **ctx.opts)
        _require_converged(info, "adjoint", ctx.opts)
        ctx.adjoint_info = info
        dvals = bkry_sddmm(ctx.h, ctx.A, lam, X, alpha=-1.0) if ctx.needs_input_grad[0] else None
        dB = lam if ctx.needs_input_grad[1] else None
        return dvals, dB, None, None, None, None, None, None, None


def block_solve(vals, B, A, h, **kw):
    """X = A(vals)^-1 B, differentiable in vals and B."""
    return BlockSolve.apply(vals, B, A, h, *[kw.get(k, d) for k, d in
                                               (("kind", "block"), ("q", 1), ("tol", 1e-13), ("maxit", 10000),
                                                ("eta", float("inf")))])
