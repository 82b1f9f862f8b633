"""Differentiable block solve X = A^-1 B for SPD A (torch.autograd.Function).

Forward: block CG on the device (bkry_cg_solve); the solution X stays on the
device for the backward pass.  Backward, for an upstream gradient G = dL/dX:
    Lambda     = A^-T G        (a second block CG solve; A^T = A for SPD A),
    dL/dB      = Lambda,
    dL/dvalues = -(Lambda X^T) on the pattern of A  (bkry_sddmm, alpha = -1).
Marshalling only: both solves and the sampled product run in the library.
"""
from __future__ import annotations

import torch


class BlockSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, B, A, h, kind="block", q=1, tol=1e-13, maxit=10000, eta=float("inf")):
        from . import CsrMatrix, bkry_cg_solve
        Av = CsrMatrix(A.n, A.rowptr, A.colind, vals.detach().contiguous())
        X, info = bkry_cg_solve(h, Av, B.detach().contiguous(), kind=kind, q=q, tol=tol, maxit=maxit, eta=eta)
        ctx.save_for_backward(X)
        ctx.A, ctx.h, ctx.opts = Av, h, dict(kind=kind, q=q, tol=tol, maxit=maxit, eta=eta)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, gX):
        from . import bkry_cg_solve, bkry_sddmm
        (X,) = ctx.saved_tensors
        lam, _ = bkry_cg_solve(ctx.h, ctx.A, gX.contiguous(), **ctx.opts)
        dvals = bkry_sddmm(ctx.h, ctx.A, lam, X, alpha=-1.0) if ctx.needs_input_grad[0] else None
        dB = lam if ctx.needs_input_grad[1] else None
        return dvals, dB, None, None, None, None, None, None, None


def block_solve(vals, B, A, h, **kw):
    """X = A(vals)^-1 B, differentiable in vals and B."""
    return BlockSolve.apply(vals, B, A, h, *[kw.get(k, d) for k, d in
                                               (("kind", "block"), ("q", 1), ("tol", 1e-13), ("maxit", 10000),
                                                ("eta", float("inf")))])
