"""Pins for the oracle's Gropp block CG (Algorithm "Gropp's BCG", Ch. 8).

Gropp's form carries Q = A P by Q = U + Q beta (U = A Z) and the
preconditioned residual by Z = Z - V lambda (V = M^-1 Q) instead of forming
A P and M^-1 R-bar anew; Ch. 8 derives it from the adaptive block CG of Ch. 4,
so in exact arithmetic its iterates are those of Ch. 4.  They are compared
with the brute-force energy minimiser over the explicit block Krylov space
(with and without a diagonal preconditioner), with textbook and scipy
(P)CG for s = 1, with the oracle's two-reduction block CG (itself pinned
independently) step by step and over whole solves -- with and without the
preconditioner, so a wrong V (M^-1 left out of the Z recurrence) or a Q
recurrence with the wrong beta fails them -- and with dense solutions.
"""
import numpy as np
import pytest

import workloads as W
from krylov_ref import galerkin_minimiser, galerkin_minimiser_prec, textbook_cg

SUBALGS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]


def small_problem(n_grid=6, s=4, seed=0):
    A = W.laplace_2d(n_grid)
    B = W.uniform_block(A.n, s, seed)
    return A, A.to_dense(), B


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_gropp_iterates_are_energy_minimisers(orc, kind, q, eta):
    A, D, B = small_problem()
    X0 = W.gaussian_block(A.n, 4, 9) * 0.1
    for k in (1, 2, 3, 4):
        r = orc.bcg_gropp(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        assert r["iters"] == k
        Xr = galerkin_minimiser(D, B, X0, k, kind, q)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-10, (k, err)


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_gropp_preconditioned_iterates_are_energy_minimisers(orc, kind, q):
    A = W.diffusion_7pt_var(4, seed=9)
    D = A.to_dense()
    minv = 1.0 / np.diag(D)
    B = W.uniform_block(A.n, 4, 0)
    X0 = W.gaussian_block(A.n, 4, 19) * 0.1
    for k in (1, 2, 3, 4):
        r = orc.bcg_gropp(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=0.0, minv=minv)
        Xr = galerkin_minimiser_prec(D, B, X0, k, kind, q, minv)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-10, (k, err)


def test_gropp_s1_is_textbook_and_scipy_pcg(orc):
    import scipy.sparse as sp
    from scipy.sparse.linalg import cg
    A, D, B = small_problem(s=1)
    for k in range(1, 9):
        r = orc.bcg_gropp(A, B, kind="block", tol=0.0, maxit=k)
        x = textbook_cg(D, B[:, 0], np.zeros(A.n), k)
        assert np.allclose(r["X"][:, 0], x, rtol=0, atol=1e-12 * np.abs(x).max())
    Av = W.diffusion_7pt_var(5, seed=10)
    Dv = Av.to_dense()
    minv = 1.0 / np.diag(Dv)
    b = W.uniform_block(Av.n, 1, 4)
    for k in (1, 2, 5, 9):
        r = orc.bcg_gropp(Av, b, kind="block", tol=0.0, maxit=k, minv=minv)
        x, _ = cg(sp.csr_matrix(Dv), b[:, 0], x0=np.zeros(Av.n), rtol=0.0, atol=0.0, maxiter=k, M=sp.diags(minv))
        assert np.allclose(r["X"][:, 0], x, rtol=0, atol=1e-11 * np.abs(x).max()), k


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, 1e4, np.inf])
def test_gropp_follows_two_reduction_bcg(orc, kind, q, eta):
    """Step by step against the two-reduction block CG (same X, residual
    history and re-normalisation decisions up to rounding), then whole
    solves (iteration and re-normalisation counts within one)."""
    A = W.laplace_2d(20)
    B = W.uniform_block(A.n, 4, 3)
    X0 = W.gaussian_block(A.n, 4, 5) * 0.01
    for k in (1, 5, 15):
        r1 = orc.bcg_gropp(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, hist_cap=k)
        r2 = orc.bcg(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, hist_cap=k)
        assert r1["iters"] == r2["iters"] == k and r1["reorth"] == r2["reorth"]
        assert np.linalg.norm(r1["X"] - r2["X"]) <= 1e-10 * np.linalg.norm(r2["X"]), k
        assert np.allclose(r1["hist"], r2["hist"], rtol=1e-8, atol=1e-15)
    r1 = orc.bcg_gropp(A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    r2 = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    assert r1["converged"] and r2["converged"]
    assert abs(r1["iters"] - r2["iters"]) <= 1
    assert abs(r1["reorth"] - r2["reorth"]) <= 1
    k = min(r1["iters"], r2["iters"]) - 1
    assert np.allclose(r1["hist"][:k], r2["hist"][:k], rtol=1e-4, atol=1e-14)


@pytest.mark.parametrize("s", [1, 2, 4])
@pytest.mark.parametrize("kind,q", SUBALGS)
def test_gropp_matches_dense_solution(orc, kind, q, s):
    if kind in ("hybrid", "bglobal") and s % 2:
        pytest.skip("q must divide s")
    A, D, B = small_problem(n_grid=10, s=s, seed=s)
    r = orc.bcg_gropp(A, B, kind=kind, q=q, tol=1e-12, maxit=1000, eta=1e4)
    assert r["converged"]
    Xs = np.linalg.solve(D, B)
    assert np.linalg.norm(r["X"] - Xs) <= 1e-9 * np.linalg.norm(Xs)
    # the recursive residual that stopped the iteration is the true one
    Rt = B - D @ r["X"]
    assert np.linalg.norm(Rt, axis=0).max() / np.linalg.norm(B, axis=0).min() < 1e-10


def test_gropp_preconditioned_full_solve(orc):
    A = W.diffusion_7pt_var(8, seed=2)
    minv = 1.0 / A.to_dense().diagonal()
    B = W.uniform_block(A.n, 4, 2)
    r1 = orc.bcg_gropp(A, B, tol=1e-10, maxit=2000, eta=1e4, minv=minv)
    r2 = orc.bcg(A, B, tol=1e-10, maxit=2000, eta=1e4, minv=minv)
    r0 = orc.bcg_gropp(A, B, tol=1e-10, maxit=2000, eta=1e4)
    assert r1["converged"] and abs(r1["iters"] - r2["iters"]) <= 1
    assert r1["iters"] < r0["iters"]
    Xs = np.linalg.solve(A.to_dense(), B)
    assert np.linalg.norm(r1["X"] - Xs) <= 1e-8 * np.linalg.norm(Xs)


def test_gropp_edge_cases(orc):
    A, D, B = small_problem(n_grid=8, s=4)
    r = orc.bcg_gropp(A, np.zeros_like(B), tol=1e-10)
    assert r["converged"] and r["iters"] == 0 and np.all(r["X"] == 0)
    assert orc.bcg_gropp(A, B, kind="hybrid", q=3)["status"] == orc.E_INVALID
    # duplicate right-hand sides: alpha is singular without re-normalisation,
    # the re-normalised iteration converges (as for the two-reduction form)
    Bd = B.copy()
    Bd[:, 2] = Bd[:, 0]
    r0 = orc.bcg_gropp(A, Bd, tol=1e-10, maxit=500, eta=0.0)
    assert r0["status"] in (orc.E_BREAKDOWN, orc.E_NONFINITE) or not r0["converged"]
    ri = orc.bcg_gropp(A, Bd, tol=1e-10, maxit=500, eta=np.inf)
    assert ri["converged"]
    assert np.linalg.norm(ri["X"] - np.linalg.solve(D, Bd)) <= 1e-8 * np.linalg.norm(np.linalg.solve(D, Bd))
    # re-normalisation counts: the initial residual and every iteration at eta = inf
    r = orc.bcg_gropp(A, B, tol=1e-10, maxit=500, eta=np.inf)
    assert r["reorth"] == r["iters"] + 1
    assert orc.bcg_gropp(A, B, tol=1e-10, maxit=500, eta=0.0)["reorth"] == 0


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, 1e4, np.inf])
def test_gropp_preconditioned_follows_two_reduction_bcg(orc, kind, q, eta):
    """With a non-trivial diagonal M the Z recurrence (Z = Z - M^-1 Q lambda)
    and the direct Z = M^-1 R-bar after a re-normalisation are both
    exercised; the iterates stay those of the preconditioned two-reduction
    block CG."""
    A = W.diffusion_7pt_var(8, seed=7)
    minv = 1.0 / A.to_dense().diagonal()
    B = W.uniform_block(A.n, 4, 8)
    for k in (1, 4, 12):
        r1 = orc.bcg_gropp(A, B, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, minv=minv, hist_cap=k)
        r2 = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, minv=minv, hist_cap=k)
        assert r1["iters"] == r2["iters"] == k and r1["reorth"] == r2["reorth"]
        assert np.linalg.norm(r1["X"] - r2["X"]) <= 1e-10 * np.linalg.norm(r2["X"]), k
        assert np.allclose(r1["hist"], r2["hist"], rtol=1e-8, atol=1e-15)
