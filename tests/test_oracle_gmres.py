"""Pins for the oracle's block Arnoldi / block GMRes (Algorithms "Block
Arnoldi Method" and "Block GMRes Method", Ch. 5).

Block GMRes minimises |B - A X|_F over X0 + K_k^S, so without restart its
k-th iterate is compared with a brute-force least-squares minimiser over an
explicitly assembled block Krylov space.  Also: the Arnoldi relation and
S-orthonormality of the basis, monotone Frobenius residual (Ch. 5,
Convergence), implicit residual = true residual, the subalgebra ordering and
the cyclic-shift example of Ch. 2 (a golden fixture).
"""
import os

import numpy as np
import pytest

import workloads as W
from krylov_ref import residual_minimiser

SUBALGS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_nonsym(N=6, s=4, seed=0):
    A = W.convdiff_2d(N, pe_h=2.0)
    B = W.gaussian_block(A.n, s, seed)
    return A, A.to_dense(), B


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_gmres_iterates_are_residual_minimisers(orc, kind, q):
    A, D, B = small_nonsym()
    X0 = W.gaussian_block(A.n, 4, 5) * 0.1
    for k in (1, 2, 3, 5):
        r = orc.bgmres(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, restart=10)
        assert r["iters"] == k and r["cycles"] == 1
        Xr = residual_minimiser(D, B, X0, k, kind, q)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-9, (k, err)


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_block_arnoldi_relation(orc, kind, q):
    A, D, B = small_nonsym(N=7)
    m = 5
    st, V, H, sig0 = orc.block_arnoldi(A, B, m, kind, q)
    assert st == 0
    assert np.allclose(V[0] @ sig0, B, atol=1e-12)
    for k in range(m):
        lhs = D @ V[k]
        rhs = sum(V[j] @ H[j, k] for j in range(k + 2))
        assert np.allclose(lhs, rhs, atol=1e-12)
    for i in range(m + 1):
        for j in range(m + 1):
            G = orc.bdot(V[i], V[j], kind, q)
            assert np.allclose(G, np.eye(4) if i == j else 0.0, atol=1e-12)


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_gmres_monotone_and_implicit_residual(orc, kind, q):
    A, D, B = small_nonsym(N=8, seed=3)
    prev = np.inf
    h = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=12, restart=12, hist_cap=12)["hist"]
    r0 = np.linalg.norm(B, axis=0)
    for k in range(1, 13):
        r = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=k, restart=12)
        R = B - D @ r["X"]
        f = np.linalg.norm(R)
        assert f <= prev * (1 + 1e-12)
        prev = f
        if kind in ("global", "bglobal"):   # Frobenius form (no per-column residual)
            assert np.isclose(h[k - 1], f / np.linalg.norm(B), rtol=1e-8)
        else:
            assert np.isclose(h[k - 1], np.max(np.linalg.norm(R, axis=0) / r0), rtol=1e-8)


def test_gmres_subalgebra_ordering(orc):
    A, D, B = small_nonsym(N=8, s=8, seed=2)
    for k in (1, 2, 4):
        res = []
        for kind, q in [("parallel", 1), ("hybrid", 4), ("hybrid", 2), ("block", 1)]:
            r = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=k, restart=10)
            res.append(np.linalg.norm(B - D @ r["X"]))
        assert all(res[i + 1] <= res[i] * (1 + 1e-10) for i in range(3)), res


def test_gmres_cyclic_shift_closed_form(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "cyclic_shift_gmres.txt")) if not l.startswith("#")]
    n = int(rows[0][0])
    D = np.roll(np.eye(n), 1, axis=1)        # ones on the superdiagonal and in the corner
    A = W.dense_to_csr(D)
    b = np.zeros((n, 1))
    b[0, 0] = 1.0
    for _, k, expect in rows:
        r = orc.bgmres(A, b, kind="block", tol=0.0, maxit=int(k), restart=n)
        got = np.linalg.norm(b - D @ r["X"])
        assert abs(got - float(expect)) < 1e-12, (k, got)
    assert np.allclose(r["X"][:, 0], np.eye(n)[1])     # the solution of the printed system is e_2


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("restart", [3, 30])
def test_gmres_restarted_matches_dense(orc, kind, q, restart):
    A, D, B = small_nonsym(N=8, seed=7)
    r = orc.bgmres(A, B, kind=kind, q=q, tol=1e-11, maxit=2000, restart=restart)
    assert r["status"] == orc.OK and r["converged"]
    Xs = np.linalg.solve(D, B)
    assert np.linalg.norm(r["X"] - Xs) / np.linalg.norm(Xs) < 1e-9
    if restart == 3:
        assert r["cycles"] > 1


def test_gmres_rank_deficient_rhs(orc):
    A, D, B = small_nonsym(N=6)
    B[:, 2] = B[:, 0]
    B[:, 3] = 0.0
    r = orc.bgmres(A, B, kind="block", tol=1e-11, maxit=500, restart=20)
    assert r["converged"]
    assert np.allclose(r["X"], np.linalg.solve(D, B), atol=1e-9)


# ---- pipelined Gram-Schmidt orthogonalisation (Ch. 9, window r) ----------
# In exact arithmetic every orthogonalisation gives the same Arnoldi basis,
# so the pipelined variants are pinned by the same independent checks as
# modified Gram-Schmidt: the residual-minimiser property of the iterates, the
# Arnoldi relation with an S-orthonormal basis, and implicit = true residual.
# A misplaced window (an update subtracted twice or not at all, an inner
# product taken before the wrong update) breaks orthogonality at the first
# step where it matters and fails the relation checks.

@pytest.mark.parametrize("r", [0, 1, 2, 3, 30])
@pytest.mark.parametrize("kind,q", SUBALGS)
def test_pipelined_gmres_iterates_are_residual_minimisers(orc, kind, q, r):
    A, D, B = small_nonsym()
    X0 = W.gaussian_block(A.n, 4, 5) * 0.1
    for k in (1, 2, 3, 5):
        res = orc.bgmres(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, restart=10, pipelined=r)
        assert res["iters"] == k and res["cycles"] == 1
        Xr = residual_minimiser(D, B, X0, k, kind, q)
        err = np.linalg.norm(res["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-9, (k, err)


@pytest.mark.parametrize("r", [1, 2, 4, 6])
@pytest.mark.parametrize("kind,q", SUBALGS)
def test_pipelined_block_arnoldi_relation(orc, kind, q, r):
    A, D, B = small_nonsym(N=7)
    m = 6
    st, V, H, sig0 = orc.block_arnoldi(A, B, m, kind, q, pipelined=r)
    assert st == 0
    assert np.allclose(V[0] @ sig0, B, atol=1e-12)
    for k in range(m):
        lhs = D @ V[k]
        rhs = sum(V[j] @ H[j, k] for j in range(k + 2))
        assert np.allclose(lhs, rhs, atol=1e-12)
    for i in range(m + 1):
        for j in range(m + 1):
            G = orc.bdot(V[i], V[j], kind, q)
            assert np.allclose(G, np.eye(4) if i == j else 0.0, atol=1e-10)


def test_pipelined_window_zero_is_modified_gram_schmidt(orc):
    """r = 0: every inner product is taken after all earlier updates, which is
    modified Gram-Schmidt operation for operation."""
    A, D, B = small_nonsym(N=8, seed=3)
    for kind, q in SUBALGS:
        a = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=14, restart=6)
        b = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=14, restart=6, pipelined=0)
        assert np.array_equal(a["X"], b["X"])


def test_pipelined_full_window_is_classical_gram_schmidt(orc):
    """r >= k: every inner product is taken with the unmodified block, i.e.
    classical Gram-Schmidt applied once; the Hessenberg column then equals
    V^T (A V_k) block by block (checked on the first steps, where the basis
    is orthonormal to rounding)."""
    A, D, B = small_nonsym(N=7)
    m = 4
    st, V, H, sig0 = orc.block_arnoldi(A, B, m, "block", 1, pipelined=m)
    assert st == 0
    for k in range(m):
        W = D @ V[k]
        for j in range(k + 1):
            assert np.allclose(H[j, k], V[j].T @ W, atol=1e-12)


def test_pipelined_gmres_converges_with_restarts(orc):
    A, D, B = small_nonsym(N=10, s=4, seed=6)
    Xs = np.linalg.solve(D, B)
    for r in (1, 3, 29):
        res = orc.bgmres(A, B, tol=1e-10, maxit=2000, restart=30, pipelined=r, hist_cap=2000)
        assert res["converged"]
        assert np.linalg.norm(res["X"] - Xs) / np.linalg.norm(Xs) < 1e-7
        assert np.all(np.diff(res["hist"][:30]) <= 1e-12)
