"""Host logic of the differentiable block solve (no GPU): an unconverged
forward or adjoint solve must raise instead of yielding wrong gradients.
The library's solver is replaced by a stand-in that reports the iteration
cap, so only the wrapper's checks run."""
import numpy as np
import pytest
import torch

import paper_2104_02494_amd as P
from paper_2104_02494_amd import autograd as AG


def _fake_solver(converged_calls):
    calls = []

    def solve(h, A, B, X=None, **kw):
        ok = converged_calls[len(calls)] if len(calls) < len(converged_calls) else True
        calls.append(kw)
        return B.clone(), dict(converged=ok, iters=kw.get("maxit"), status=0 if ok else 1)
    return solve, calls


def _problem():
    n = 4
    rowptr = torch.tensor([0, 1, 2, 3, 4], dtype=torch.int32)
    colind = torch.arange(n, dtype=torch.int32)
    A = P.CsrMatrix(n, rowptr, colind, torch.full((n,), 2.0, dtype=torch.float64))
    vals = torch.full((n,), 2.0, dtype=torch.float64, requires_grad=True)
    B = torch.ones(n, 2, dtype=torch.float64, requires_grad=True)
    return A, vals, B


def test_forward_not_converged_raises(monkeypatch):
    solve, calls = _fake_solver([False])
    monkeypatch.setattr(P, "bkry_cg_solve", solve)
    A, vals, B = _problem()
    with pytest.raises(AG.SolveNotConverged, match="forward"):
        AG.block_solve(vals, B, A, None, maxit=3)
    assert len(calls) == 1 and calls[0]["maxit"] == 3


def test_adjoint_not_converged_raises(monkeypatch):
    solve, calls = _fake_solver([True, False])
    monkeypatch.setattr(P, "bkry_cg_solve", solve)
    monkeypatch.setattr(P, "bkry_sddmm", lambda *a, **k: torch.zeros(4, dtype=torch.float64))
    A, vals, B = _problem()
    X = AG.block_solve(vals, B, A, None, maxit=3)
    with pytest.raises(AG.SolveNotConverged, match="adjoint"):
        X.sum().backward()
    assert len(calls) == 2


def test_converged_solves_give_gradients(monkeypatch):
    solve, calls = _fake_solver([True, True])
    monkeypatch.setattr(P, "bkry_cg_solve", solve)
    monkeypatch.setattr(P, "bkry_sddmm", lambda h, A, lam, X, alpha: alpha * (lam * X).sum(1))
    A, vals, B = _problem()
    X = AG.block_solve(vals, B, A, None)
    X.sum().backward()
    assert np.array_equal(B.grad.numpy(), np.ones((4, 2)))
    assert np.array_equal(vals.grad.numpy(), -2.0 * np.ones(4))
