"""Pins for the oracle's block CG (Algorithm "BCG Method with Adaptive
Residual Re-Orthonormalization", Ch. 4).

The block CG iterate X^k is the energy minimiser over X0 + K_k^S (Theorem
"minimizing-orthogonality", Ch. 4), so it is compared with a brute-force
minimiser over an explicitly assembled block Krylov space; s = 1 and the
parallel subalgebra reduce to textbook scalar CG, global to scalar CG on the
Kronecker system (Definition "elementary *-subalgebras"); plus finite
termination, orthogonality invariants, the subalgebra-lattice ordering
(Lemma "Embeddings of *-subalgebras"), the eigenvector one-step case and the
Chebyshev bound (Ch. 2 / Ch. 4 convergence results).
"""
import numpy as np
import pytest

import workloads as W
from krylov_ref import (energy_fro, galerkin_minimiser, galerkin_minimiser_prec, laplace2d_eigpair,
                        laplace2d_extremes, textbook_cg)

SUBALGS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]


def small_problem(n_grid=6, s=4, seed=0):
    A = W.laplace_2d(n_grid)
    B = W.uniform_block(A.n, s, seed)
    return A, A.to_dense(), B


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_bcg_iterates_are_energy_minimisers(orc, kind, q, eta):
    A, D, B = small_problem()
    X0 = W.gaussian_block(A.n, 4, 9) * 0.1
    for k in (1, 2, 3, 4):
        r = orc.bcg(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        assert r["iters"] == k
        Xr = galerkin_minimiser(D, B, X0, k, kind, q)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-10, (k, err)


def test_bcg_s1_is_textbook_cg(orc):
    A, D, B = small_problem(s=1)
    for k in range(1, 9):
        r = orc.bcg(A, B, kind="block", tol=0.0, maxit=k)
        x = textbook_cg(D, B[:, 0], np.zeros(A.n), k)
        assert np.allclose(r["X"][:, 0], x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_bcg_parallel_is_independent_cgs(orc):
    A, D, B = small_problem(s=5)
    for k in (1, 3, 7, 12):
        r = orc.bcg(A, B, kind="parallel", tol=0.0, maxit=k)
        for j in range(5):
            x = textbook_cg(D, B[:, j], np.zeros(A.n), k)
            assert np.allclose(r["X"][:, j], x, rtol=0, atol=1e-11 * np.abs(x).max())


def test_bcg_global_is_cg_on_kronecker_system(orc):
    A, D, B = small_problem(s=3)
    Dk = np.kron(np.eye(3), D)
    for k in (1, 2, 5, 9):
        r = orc.bcg(A, B, kind="global", tol=0.0, maxit=k)
        x = textbook_cg(Dk, B.reshape(-1, order="F"), np.zeros(3 * A.n), k)
        assert np.allclose(r["X"].reshape(-1, order="F"), x, rtol=0, atol=1e-11 * np.abs(x).max())


def test_bcg_hybrid_is_independent_block_solves(orc):
    A, D, B = small_problem(s=8)
    for k in (1, 3, 6):
        r = orc.bcg(A, B, kind="hybrid", q=2, tol=0.0, maxit=k)
        for grp in range(2):
            sub = orc.bcg(A, B[:, 4 * grp:4 * grp + 4], kind="block", tol=0.0, maxit=k)
            assert np.allclose(r["X"][:, 4 * grp:4 * grp + 4], sub["X"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2, 4])
@pytest.mark.parametrize("kind,q", SUBALGS)
def test_bcg_matches_dense_solution(orc, kind, q, s):
    if kind in ("hybrid", "bglobal") and s % 2:
        pytest.skip("q must divide s")
    grid = small_problem(n_grid=7, s=s, seed=s)
    A2 = W.random_spd_csr(60, 0.1, seed=s, shift=1.0)
    rnd = (A2, A2.to_dense(), W.uniform_block(60, s, s))
    for (A, D, B), eta in [(grid, np.inf), (rnd, 1e4), (rnd, 0.0)]:
        r = orc.bcg(A, B, kind=kind, q=q, tol=1e-12, maxit=500, eta=eta)
        assert r["status"] == orc.OK and r["converged"]
        Xs = np.linalg.solve(D, B)
        assert np.linalg.norm(r["X"] - Xs) / np.linalg.norm(Xs) < 1e-10
        R = B - D @ r["X"]
        assert np.all(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0) < 1e-11)


def test_bcg_exhausted_krylov_space_breaks_down_without_reortho(orc):
    """The 7x7 grid Laplacian has repeated eigenvalues, so the block Krylov
    space is exhausted before ceil(n/s) steps and the residual turns rank
    deficient; with eta = 0 (and here also eta = 1e4, whose kappa_D test does
    not fire in time) the Cholesky of rho fails, while eta = inf converges."""
    A, D, B = small_problem(n_grid=7, s=4, seed=4)
    assert orc.bcg(A, B, kind="block", tol=1e-12, maxit=500, eta=0.0)["status"] == orc.E_BREAKDOWN
    r = orc.bcg(A, B, kind="block", tol=1e-12, maxit=500, eta=np.inf)
    assert r["converged"] and r["iters"] <= 13


@pytest.mark.parametrize("kind,q,g", [("block", 1, 4), ("hybrid", 2, 2), ("parallel", 1, 1)])
def test_bcg_finite_termination(orc, kind, q, g):
    """X* lies in X0 + K_nu with block grade nu <= ceil(n/g) (Lemma on the block grade, Ch. 3)."""
    A = W.random_spd_csr(24, 0.2, seed=4, shift=2.0)
    B = W.gaussian_block(24, 4, 1)
    r = orc.bcg(A, B, kind=kind, q=q, tol=1e-8, maxit=200, eta=np.inf)
    assert r["converged"] and r["iters"] <= int(np.ceil(24 / g))


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_bcg_orthogonality_invariants(orc, kind, q):
    """<R^k, P^j>_S = 0 for j < k and <P^i, A P^j>_S = 0 for i != j."""
    A, D, B = small_problem(n_grid=8, s=4)
    r = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=5, eta=1e4, record_blocks=6)
    Pk, Rk = r["Pk"], r["Rk"]
    for k in range(len(Rk)):
        for j in range(k):
            G = orc.bdot(Rk[k], Pk[j], kind, q)
            assert np.abs(G).max() < 1e-11 * np.linalg.norm(Rk[k]) * np.linalg.norm(Pk[j])
    for i in range(len(Pk)):
        for j in range(len(Pk)):
            if i != j:
                G = orc.bdot(Pk[i], D @ Pk[j], kind, q)
                scale = np.linalg.norm(Pk[i]) * np.linalg.norm(D @ Pk[j])
                assert np.abs(G).max() < 1e-11 * scale


def test_bcg_lattice_ordering(orc):
    """Energy errors at equal k are ordered S_P >= S_BP^2 >= S_BP^4 >= S_B."""
    A, D, B = small_problem(n_grid=8, s=8, seed=3)
    Xs = np.linalg.solve(D, B)
    for k in (1, 2, 3, 4):
        errs = []
        for kind, q in [("parallel", 1), ("hybrid", 4), ("hybrid", 2), ("block", 1)]:
            r = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=k)
            errs.append(energy_fro(D, r["X"] - Xs))
        assert all(errs[i + 1] <= errs[i] * (1 + 1e-10) for i in range(3)), errs


@pytest.mark.parametrize("kind", ["block", "parallel"])
def test_bcg_eigenvector_rhs_one_step(orc, kind):
    N = 8
    pairs = [laplace2d_eigpair(N, i, j) for (i, j) in [(1, 1), (1, 2), (2, 3), (4, 1)]]
    B = np.stack([u for _, u in pairs], axis=1)
    A = W.laplace_2d(N)
    r = orc.bcg(A, B, kind=kind, tol=1e-12, maxit=10)
    assert r["converged"] and r["iters"] == 1
    Xs = B / np.array([lam for lam, _ in pairs])[None, :]
    assert np.allclose(r["X"], Xs, atol=1e-13)


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_bcg_chebyshev_bound(orc, kind, q):
    N = 10
    A = W.laplace_2d(N)
    D = A.to_dense()
    B = W.uniform_block(A.n, 4, 2)
    lo, hi = laplace2d_extremes(N)
    kap = hi / lo
    mu = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    Xs = np.linalg.solve(D, B)
    e0 = energy_fro(D, Xs)
    for k in (1, 5, 10, 20):
        r = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=k)
        assert energy_fro(D, r["X"] - Xs) <= 2 * mu ** k * e0 * (1 + 1e-12)


def test_bcg_breakdown_and_edge_cases(orc):
    A, D, B = small_problem()
    negA = W.Csr(A.n, A.rowptr, A.colind, -A.val)
    assert orc.bcg(negA, B, kind="block", eta=0.0)["status"] == orc.E_BREAKDOWN
    Bz = B.copy()
    Bz[:, 1] = 0.0
    assert orc.bcg(A, Bz, kind="block", eta=0.0, tol=1e-12)["status"] == orc.E_BREAKDOWN
    r = orc.bcg(A, Bz, kind="block", eta=np.inf, tol=1e-12, maxit=200)
    assert r["converged"] and np.abs(r["X"][:, 1]).max() < 1e-12
    assert np.allclose(r["X"], np.linalg.solve(D, Bz), atol=1e-10)
    r = orc.bcg(A, np.zeros_like(B), kind="block")
    assert r["converged"] and r["iters"] == 0 and np.all(r["X"] == 0)
    r = orc.bcg(A, B, kind="block", maxit=1, tol=1e-10)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 1
    assert orc.bcg(A, B, kind="hybrid", q=3)["status"] == orc.E_INVALID


def test_bcg_reortho_counts(orc):
    A, D, B = small_problem(n_grid=10, s=4)
    r = orc.bcg(A, B, kind="block", tol=1e-10, maxit=500, eta=np.inf)
    assert r["reorth"] == r["iters"] + 1       # the initial residual and every iteration
    r0 = orc.bcg(A, B, kind="block", tol=1e-10, maxit=500, eta=0.0)
    assert r0["reorth"] == 0
    rp = orc.bcg(A, B, kind="parallel", tol=1e-10, maxit=500, eta=1e4)
    assert rp["reorth"] == 1                  # kappa_D = 1 in the parallel case


def test_bcg_recursive_residual_tracks_true_residual(orc):
    A, D, B = small_problem(n_grid=12, s=4)
    for eta in (0.0, 1e4, np.inf):
        r = orc.bcg(A, B, kind="block", tol=1e-10, maxit=500, eta=eta)
        true = np.linalg.norm(B - D @ r["X"], axis=0) / np.linalg.norm(B, axis=0)
        assert np.allclose(true, r["relres"], rtol=1e-3, atol=1e-13)
        assert r["relres"].max() <= 1e-10


# ------------------------------------------------ diagonal preconditioner --
def prec_problem(N=4, s=4, seed=0):
    """Variable-coefficient 7-point diffusion (diagonal far from constant)
    with the Jacobi preconditioner M = diag(A)."""
    A = W.diffusion_7pt_var(N, seed=5 + N)
    D = A.to_dense()
    minv = 1.0 / np.diag(D)
    B = W.uniform_block(A.n, s, seed)
    return A, D, B, minv


@pytest.mark.parametrize("kind,q", SUBALGS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_pbcg_iterates_are_energy_minimisers(orc, kind, q, eta):
    """With M != I the k-th iterate minimises the A-energy error over
    X0 + K_k^S(M^-1 A, M^-1 R0)."""
    A, D, B, minv = prec_problem()
    assert np.ptp(minv) > 0.5 * minv.max()       # a genuinely non-constant M
    X0 = W.gaussian_block(A.n, 4, 19) * 0.1
    for k in (1, 2, 3, 4):
        r = orc.bcg(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta, minv=minv)
        assert r["iters"] == k
        Xr = galerkin_minimiser_prec(D, B, X0, k, kind, q, minv)
        err = np.linalg.norm(r["X"] - Xr) / np.linalg.norm(Xr)
        assert err < 1e-10, (k, err)
        # and it is not the unpreconditioned iterate
        if k > 1:
            assert np.linalg.norm(r["X"] - galerkin_minimiser(D, B, X0, k, kind, q)) > 1e-6 * np.linalg.norm(Xr)


def test_pbcg_s1_and_parallel_are_scipy_pcg(orc):
    """s = 1 and the parallel subalgebra reduce to textbook preconditioned CG
    (scipy.sparse.linalg.cg with M = diag(minv)), column by column."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import cg
    A, D, B, minv = prec_problem(N=5, s=3)
    As, Ms = sp.csr_matrix(D), sp.diags(minv)
    for k in (1, 2, 5, 9):
        r1 = orc.bcg(A, B[:, :1], kind="block", tol=0.0, maxit=k, minv=minv)
        rp = orc.bcg(A, B, kind="parallel", tol=0.0, maxit=k, minv=minv)
        for j in range(3):
            x, _ = cg(As, B[:, j], x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=k, M=Ms)
            sc = np.abs(x).max()
            assert np.allclose(rp["X"][:, j], x, rtol=0, atol=1e-11 * sc), (k, j)
            if j == 0:
                assert np.allclose(r1["X"][:, 0], x, rtol=0, atol=1e-11 * sc), k


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_pbcg_power_of_two_scalar_preconditioner_is_exact(orc, kind, q):
    """M^-1 = c I with c a power of two scales P, rho and alpha by exact
    powers of two that cancel in lambda sigma and beta: the iterates equal
    the unpreconditioned ones bit for bit (a misplaced M^-1, e.g. in rho,
    leaves a factor c in lambda)."""
    A, D, B = small_problem(n_grid=6, s=4, seed=4)
    for eta in (0.0, 1e4, np.inf):
        r0 = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=200, eta=eta)
        r1 = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=200, eta=eta, minv=np.full(A.n, 0.25))
        assert r0["iters"] == r1["iters"] and r0["reorth"] == r1["reorth"]
        assert np.array_equal(r0["X"], r1["X"])


@pytest.mark.parametrize("kind,q", SUBALGS)
def test_pbcg_orthogonality_invariants(orc, kind, q):
    """<R^k, P^j>_S = 0 (j < k), <P^i, A P^j>_S = 0 (i != j) and the
    preconditioned residuals are conjugate to the residuals:
    <M^-1 R^i, R^j>_S = 0 (i != j)."""
    A, D, B, minv = prec_problem(N=5, s=4)
    r = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=5, eta=1e4, record_blocks=6, minv=minv)
    Pk, Rk = r["Pk"], r["Rk"]
    for k in range(len(Rk)):
        for j in range(k):
            G = orc.bdot(Rk[k], Pk[j], kind, q)
            assert np.abs(G).max() < 1e-11 * np.linalg.norm(Rk[k]) * np.linalg.norm(Pk[j])
            Z = orc.bdot(minv[:, None] * Rk[j], Rk[k], kind, q)
            assert np.abs(Z).max() < 1e-11 * np.linalg.norm(minv[:, None] * Rk[j]) * np.linalg.norm(Rk[k])
    for i in range(len(Pk)):
        for j in range(len(Pk)):
            if i != j:
                G = orc.bdot(Pk[i], D @ Pk[j], kind, q)
                assert np.abs(G).max() < 1e-11 * np.linalg.norm(Pk[i]) * np.linalg.norm(D @ Pk[j])


def test_pbcg_exact_preconditioner_converges_in_one_step(orc):
    """A diagonal, M = A: M^-1 A = I, so one block iteration is exact."""
    n = 50
    d = np.linspace(1.0, 100.0, n)
    A = W.dense_to_csr(np.diag(d))
    B = W.uniform_block(n, 4, 2)
    for kind, q in SUBALGS:
        r = orc.bcg(A, B, kind=kind, q=q, tol=1e-12, maxit=5, minv=1.0 / d)
        assert r["converged"] and r["iters"] == 1
        assert np.allclose(r["X"], B / d[:, None], rtol=1e-12, atol=0)


# --------------------------------------------------- block-global subalgebra --
def test_block_global_inner_product_and_normaliser(orc):
    """S_BG(q) (Definition "Relevant *-subalgebras", Ch. 3): <X, Y> =
    (1/q) sum_i I_q (x) X_i^T Y_i; the normaliser is the QR of the stacked
    groups, N = I_q (x) rho / sqrt(q), Y = sqrt(q) Y~ (example "Normalizer in
    the block-global *-subalgebra"), checked against numpy's QR."""
    X = W.gaussian_block(300, 8, 31)
    Y = W.gaussian_block(300, 8, 32)
    for q in (2, 4):
        g = 8 // q
        mean = sum(X[:, i * g:(i + 1) * g].T @ Y[:, i * g:(i + 1) * g] for i in range(q)) / q
        assert np.allclose(orc.bdot(X, Y, "bglobal", q), np.kron(np.eye(q), mean), rtol=1e-13, atol=1e-13)
        Yn, N = orc.normalize(X, "bglobal", q)
        stacked = np.vstack([X[:, i * g:(i + 1) * g] for i in range(q)])
        _, rho = np.linalg.qr(stacked)
        rho = rho * np.sign(np.diag(rho))[:, None]
        assert np.allclose(N, np.kron(np.eye(q), rho / np.sqrt(q)), rtol=1e-12, atol=1e-12)
        assert np.allclose(orc.bdot(Yn, Yn, "bglobal", q), np.eye(8), atol=1e-13)
        assert np.allclose(Yn @ N, X, atol=1e-12)


def test_block_global_lattice(orc):
    """S_G subset S_BG(q) subset S_B (Lemma "Embeddings of *-subalgebras"):
    the block Krylov spaces are nested, so the energy errors at equal k are
    ordered global >= block-global >= block."""
    A, D, B = small_problem(n_grid=8, s=8, seed=5)
    Xs = np.linalg.solve(D, B)
    for k in (2, 4, 6):
        e = {}
        for kind, q in (("global", 1), ("bglobal", 2), ("block", 1)):
            r = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=k, eta=np.inf)
            e[kind] = energy_fro(D, r["X"] - Xs)
        assert e["global"] >= e["bglobal"] * (1 - 1e-10) >= e["block"] * (1 - 1e-10), (k, e)
