"""Pins for the oracle's multicolour SSOR preconditioner and the block CG it
preconditions (Algorithm "BCG Method with Adaptive Residual
Re-Orthonormalization", Ch. 4, with an SSOR-type M as in the experiments).

The colouring is pinned by its defining property (every row holds the
smallest colour that no higher-priority neighbour holds), its validity and,
for the natural order on a grid, the closed-form checkerboard; the sweeps by
the SSOR matrix written out densely from its definition, its symmetry and
the one-colour case; the preconditioned CG by the brute-force energy
minimiser over K_k^S(M^-1 A, M^-1 R0), scipy's PCG with the same M for
s = 1, and dense solutions.
"""
import numpy as np
import pytest

import workloads as W
from krylov_ref import galerkin_minimiser_precmat, ssor_matrix

SUBALGS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]


def neighbours(A, i):
    return [j for j in A.colind[A.rowptr[i]:A.rowptr[i + 1]] if j != i]


@pytest.mark.parametrize("name", ["lap2d", "lap3d", "diff27", "randspd"])
def test_coloring_is_greedy_in_priority_order(orc, name):
    A = {"lap2d": lambda: W.laplace_2d(13), "lap3d": lambda: W.laplace_3d(7),
         "diff27": lambda: W.diffusion_27pt(5, seed=4),
         "randspd": lambda: W.random_spd_csr(300, 0.03, seed=5)}[name]()
    prio = W.color_priorities(A.n, 11)
    prio[::7] = prio[3]                               # ties, broken by the row index
    colors, nc = orc.color_greedy(A, prio)
    assert nc == colors.max() + 1 and colors.min() == 0
    beats = lambda u, v: prio[u] > prio[v] or (prio[u] == prio[v] and u < v)
    for v in range(A.n):
        nb = neighbours(A, v)
        assert all(colors[u] != colors[v] for u in nb)                  # valid
        taken = {colors[u] for u in nb if beats(u, v)}
        mex = next(c for c in range(len(nb) + 2) if c not in taken)
        assert colors[v] == mex                                         # greedy in priority order
    assert nc <= max(len(neighbours(A, v)) for v in range(A.n)) + 1


@pytest.mark.parametrize("dims", [2, 3])
def test_coloring_natural_order_is_checkerboard(orc, dims):
    N = 9
    A = W.laplace_2d(N) if dims == 2 else W.laplace_3d(N)
    prio = (A.n - 1 - np.arange(A.n)).astype(np.uint32)             # row 0 first
    colors, nc = orc.color_greedy(A, prio)
    idx = np.arange(A.n)
    parity = sum((idx // N ** d) % N for d in range(dims)) % 2
    assert nc == 2 and np.array_equal(colors, parity)


@pytest.mark.parametrize("omega", [1.0, 1.5, 0.7])
@pytest.mark.parametrize("name", ["var7", "diff27"])
def test_ssor_apply_is_the_ssor_matrix_inverse(orc, omega, name):
    A = W.diffusion_7pt_var(6, seed=3) if name == "var7" else W.diffusion_27pt(5, seed=6)
    D = A.to_dense()
    colors, nc = orc.color_greedy(A, W.color_priorities(A.n, 2))
    assert nc >= 2
    R = W.gaussian_block(A.n, 3, 4)
    st, Z = orc.ssor_apply(A, colors, omega, R)
    assert st == orc.OK
    M = ssor_matrix(D, colors, omega)
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())   # symmetric for symmetric A
    Zr = np.linalg.solve(M, R)
    assert np.abs(Z - Zr).max() <= 1e-12 * np.abs(Zr).max()
    # M^-1 is symmetric positive definite: v^T M^-1 w = w^T M^-1 v, v^T M^-1 v > 0
    v, w = R[:, 0], R[:, 1]
    _, Mv = orc.ssor_apply(A, colors, omega, v[:, None])
    _, Mw = orc.ssor_apply(A, colors, omega, w[:, None])
    assert abs(w @ Mv[:, 0] - v @ Mw[:, 0]) <= 1e-12 * np.abs(Mv).max() * np.abs(w).sum()
    assert v @ Mv[:, 0] > 0


def test_ssor_one_colour_and_errors(orc):
    # a diagonal matrix: one colour, M = D / (omega (2 - omega))
    d = np.linspace(1.0, 3.0, 20)
    A = W.dense_to_csr(np.diag(d))
    colors, nc = orc.color_greedy(A, W.color_priorities(A.n, 1))
    assert nc == 1
    R = W.gaussian_block(A.n, 2, 5)
    st, Z = orc.ssor_apply(A, colors, 1.3, R)
    assert st == orc.OK and np.allclose(Z, 1.3 * 0.7 * R / d[:, None], rtol=1e-14, atol=0)
    # two coupled rows of one colour, and a row without a positive diagonal
    L = W.laplace_2d(5)
    assert orc.ssor_apply(L, np.zeros(L.n, dtype=np.int32), 1.0, R[:L.n] if L.n <= 20 else
                          W.gaussian_block(L.n, 2, 1))[0] == orc.E_INVALID
    negL = W.Csr(L.n, L.rowptr, L.colind, -L.val)
    c, _ = orc.color_greedy(L, W.color_priorities(L.n, 3))
    assert orc.ssor_apply(negL, c, 1.0, W.gaussian_block(L.n, 2, 1))[0] == orc.E_INVALID


def ssor_problem(N=4, s=4, seed=0, omega=1.2):
    A = W.diffusion_7pt_var(N, seed=5 + N)
    colors, _ = orc_colors(A)
    return A, A.to_dense(), W.uniform_block(A.n, s, seed), colors, omega


def orc_colors(A):
    import oracle
    return oracle.color_greedy(A, W.color_priorities(A.n, 17))


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_ssor_pcg_iterates_are_energy_minimisers(orc, kind, q, eta):
    A, D, B, colors, omega = ssor_problem()
    Minv = np.linalg.inv(ssor_matrix(D, colors, omega))
    X0 = W.gaussian_block(A.n, 4, 19) * 0.1
    for k in (1, 2, 3, 4):
        r = orc.bcg_ssor(A, B, colors, omega, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        assert r["iters"] == k
        Xr = galerkin_minimiser_precmat(D, B, X0, k, kind, q, Minv)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-10, (k, err)


def test_ssor_pcg_s1_is_scipy_pcg(orc):
    import scipy.sparse as sp
    from scipy.sparse.linalg import LinearOperator, cg
    A, D, B, colors, omega = ssor_problem(N=5, s=1, omega=1.0)
    Minv = np.linalg.inv(ssor_matrix(D, colors, omega))
    Mop = LinearOperator(D.shape, matvec=lambda v: Minv @ v)
    for k in (1, 2, 5, 9):
        r = orc.bcg_ssor(A, B, colors, omega, tol=0.0, maxit=k)
        x, _ = cg(sp.csr_matrix(D), B[:, 0], x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=k, M=Mop)
        assert np.allclose(r["X"][:, 0], x, rtol=0, atol=1e-11 * np.abs(x).max()), k


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_ssor_pcg_full_solve(orc, kind, q):
    A = W.diffusion_7pt_var(8, seed=2)
    D = A.to_dense()
    B = W.uniform_block(A.n, 4, 2)
    colors, _ = orc_colors(A)
    r = orc.bcg_ssor(A, B, colors, 1.0, kind=kind, q=q, tol=1e-10, maxit=2000, eta=1e4)
    rj = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=1e4, minv=1.0 / np.diag(D))
    assert r["converged"] and r["iters"] < rj["iters"]
    Xs = np.linalg.solve(D, B)
    assert np.linalg.norm(r["X"] - Xs) <= 1e-8 * np.linalg.norm(Xs)
    assert orc.bcg_ssor(A, B, np.zeros(A.n, dtype=np.int32), 1.0)["status"] == orc.E_INVALID
