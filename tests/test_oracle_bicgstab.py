"""Pins for the oracle's block BiCGStab with adaptive residual
re-orthonormalisation (Algorithm "BBiCGStab with Adaptive Residual
Re-Orthonormalization", Ch. 6) and its coefficient solves.

s = 1 without re-orthonormalisation reduces to the textbook BiCGStab of van
der Vorst (scipy.sparse.linalg.bicgstab with the shadow residual r0); the
recursive residual R^ sigma must equal the true residual B - A X after any
number of steps (it fails if an X update uses the wrong transformation
sigma after a re-normalisation); converged solutions match a dense solve;
the per-S-block LU solve matches numpy."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import bicgstab

import workloads as W

SUBALGS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]


def test_lu_solve_matches_numpy(orc):
    rng = np.random.default_rng(1)
    s = 8
    A = rng.standard_normal((s, s)) + 0.1 * np.eye(s)
    B = rng.standard_normal((s, s))
    st, X = orc.lu_solve(A, B, "block")
    assert st == 0 and np.allclose(X, np.linalg.solve(A, B), rtol=1e-12, atol=1e-12)
    # hybrid: block-diagonal parts only
    st, X = orc.lu_solve(A, B, "hybrid", 2)
    ref = np.zeros((s, s))
    for o in (0, 4):
        ref[o:o + 4, o:o + 4] = np.linalg.solve(A[o:o + 4, o:o + 4], B[o:o + 4, o:o + 4])
    assert st == 0 and np.allclose(X, ref, rtol=1e-12, atol=1e-12)
    # a matrix that needs row exchanges (zero leading entry)
    P = np.eye(s)[::-1] + 0.01 * rng.standard_normal((s, s))
    P[0, 0] = 0.0
    st, X = orc.lu_solve(P, B, "block")
    assert st == 0 and np.allclose(P @ X, B, atol=1e-10)
    st, _ = orc.lu_solve(np.zeros((s, s)), B, "block")
    assert st == -2


def test_s1_is_textbook_bicgstab(orc):
    A = W.convdiff_2d(14)
    D = sp.csr_matrix(A.to_dense())
    b = W.gaussian_block(A.n, 1, 3)
    for k in (1, 2, 4, 8):                           # rounding grows with k on this non-normal A
        r = orc.bbicgstab(A, b, kind="block", tol=0.0, maxit=k, eta=0.0)
        x, _ = bicgstab(D, b[:, 0], x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=k)
        assert r["iters"] == k
        assert np.abs(r["X"][:, 0] - x).max() <= 1e-12 * np.abs(x).max(), k


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, 1e4, np.inf])
def test_recursive_residual_is_true_residual(orc, kind, q, eta):
    A = W.convdiff_2d(12)
    D = A.to_dense()
    B = W.gaussian_block(A.n, 4, 11)
    r0 = np.linalg.norm(B, axis=0)
    for k in (1, 3, 6):
        r = orc.bbicgstab(A, B, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, hist_cap=k)
        true = np.linalg.norm(B - D @ r["X"], axis=0) / r0
        assert np.allclose(true, r["relres"], rtol=1e-8, atol=1e-13), (k, true, r["relres"])
        if eta == np.inf:
            assert r["reorth"] == k + 1


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_converges_to_dense_solution(orc, kind, q, eta):
    A = W.convdiff_2d(16)
    D = A.to_dense()
    B = W.gaussian_block(A.n, 4, 12)
    r = orc.bbicgstab(A, B, kind=kind, q=q, tol=1e-10, maxit=1000, eta=eta)
    assert r["converged"]
    Xs = np.linalg.solve(D, B)
    assert np.linalg.norm(r["X"] - Xs) <= 1e-6 * np.linalg.norm(Xs)


def test_edge_cases(orc):
    A = W.convdiff_2d(8)
    B = W.gaussian_block(A.n, 4, 2)
    r = orc.bbicgstab(A, np.zeros_like(B), tol=1e-10)
    assert r["converged"] and r["iters"] == 0 and np.all(r["X"] == 0)
    n = 40
    I = W.dense_to_csr(np.eye(n) * 3.0)
    Bi = W.gaussian_block(n, 4, 1)
    r = orc.bbicgstab(I, Bi, tol=1e-12, maxit=5)       # A = 3 I: exact after one step
    assert r["converged"] and r["iters"] == 1 and np.allclose(r["X"], Bi / 3.0, rtol=1e-13)
    # duplicate right-hand sides: a rank-deficient block.  Without
    # re-orthonormalisation the coefficient system is singular (breakdown or
    # no convergence); with it the solve converges
    Bd = B.copy()
    Bd[:, 1] = Bd[:, 0]
    r = orc.bbicgstab(A, Bd, tol=1e-10, maxit=500, eta=np.inf)
    assert r["converged"]
    r0 = orc.bbicgstab(A, Bd, tol=1e-10, maxit=500, eta=0.0)
    assert r0["status"] != 0


# ---- restart on the true residual (reading beyond the listing) -----------
def test_restarted_bicgstab_closes_the_residual_gap(orc):
    """On the 128^2 convection-diffusion problem the plain iteration stops at
    1e-10 on its recursive residual with a true residual near 2.5e-8; the
    restarted one continues from that iterate until the true residual,
    recomputed here with numpy, meets 1e-10."""
    A = W.convdiff_2d(128)
    B = W.gaussian_block(A.n, 8, 1004)
    M = sp.csr_matrix((A.val, A.colind, A.rowptr), shape=(A.n, A.n))
    plain = orc.bbicgstab(A, B, tol=1e-10, maxit=5000, eta=1e4)
    true_plain = np.linalg.norm(B - M @ plain["X"], axis=0) / np.linalg.norm(B, axis=0)
    assert plain["converged"] and true_plain.max() > 1e-10
    r = orc.bbicgstab(A, B, tol=1e-10, maxit=5000, eta=1e4, max_restarts=10)
    true_r = np.linalg.norm(B - M @ r["X"], axis=0) / np.linalg.norm(B, axis=0)
    assert r["converged"] and r["restarts"] >= 1
    assert true_r.max() <= 1e-10
    assert np.allclose(r["relres"], true_r, rtol=1e-6, atol=1e-16)
    assert r["iters"] > plain["iters"]


def test_restarted_bicgstab_without_restarts_is_the_plain_iteration(orc):
    A = W.convdiff_2d(24)
    B = W.gaussian_block(A.n, 4, 9)
    for kind, q in SUBALGS:
        a = orc.bbicgstab(A, B, kind=kind, q=q, tol=0.0, maxit=12, eta=1e4)
        b = orc.bbicgstab(A, B, kind=kind, q=q, tol=0.0, maxit=12, eta=1e4, max_restarts=3)
        assert np.array_equal(a["X"], b["X"]) and b["restarts"] == 0 and b["iters"] == 12
        c = orc.bbicgstab(A, B, kind=kind, q=q, tol=1e-10, maxit=1000, eta=1e4, max_restarts=0)
        d = orc.bbicgstab(A, B, kind=kind, q=q, tol=1e-10, maxit=1000, eta=1e4)
        assert np.array_equal(c["X"], d["X"]) and c["iters"] == d["iters"]
        true_c = np.linalg.norm(B - A.to_dense() @ c["X"], axis=0) / np.linalg.norm(B, axis=0)
        assert c["converged"] == bool(true_c.max() <= 1e-10)


def test_restarted_bicgstab_respects_the_iteration_budget(orc):
    A = W.convdiff_2d(64)
    B = W.gaussian_block(A.n, 4, 11)
    r = orc.bbicgstab(A, B, tol=1e-14, maxit=150, eta=1e4, max_restarts=50)
    assert r["iters"] <= 150 and not r["converged"]
