"""Pins for the oracle's building blocks (BOP/SpMM, BDOT, projections,
Householder normaliser, Cholesky solves in S, kappa_D, SDDMM, CSR transpose).

Each oracle function is compared with something independent of it: dense numpy
or scipy linear algebra, integer-valued inputs whose result is exact in any
summation order, the axioms of a block inner product (Definition "block inner
product", Ch. 3) and the defining properties of a normaliser (Definition
"normalizer", Ch. 3).
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse

import workloads as W

KINDS = [("block", 1), ("hybrid", 2), ("hybrid", 4), ("parallel", 1), ("global", 1)]


def s_mask(s, kind, q):
    """Sparsity pattern of the subalgebra (Definitions of S_G, S_P, S_B, S_BP)."""
    if kind == "block":
        return np.ones((s, s), bool)
    if kind in ("parallel", "global"):
        return np.eye(s, dtype=bool)
    g = s // q
    idx = np.arange(s) // g
    return idx[:, None] == idx[None, :]


def random_in_S(rng, s, kind, q):
    if kind == "global":
        return rng.standard_normal() * np.eye(s)
    return np.where(s_mask(s, kind, q), rng.standard_normal((s, s)), 0.0)


# ----------------------------------------------------------------- SpMM ----
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8, 16, 32])
def test_spmm_integer_exact(orc, s):
    A = W.random_csr(97, 97, 0.1, seed=s, integer=True, empty_rows=(0, 13, 96))
    X = np.random.default_rng(s).integers(-8, 9, size=(97, s)).astype(float)
    Y = orc.spmm(A, X)
    assert np.array_equal(Y, A.to_dense() @ X)          # integer sums are exact in any order
    assert np.all(Y[[0, 13, 96]] == 0.0)


def test_spmm_random_matches_dense(orc):
    A = W.laplace_3d(6)
    X = W.gaussian_block(A.n, 8, 3)
    ref = A.to_dense() @ X
    assert np.allclose(orc.spmm(A, X), ref, rtol=0, atol=1e-13)


# ----------------------------------------------------------------- BDOT ----
@pytest.mark.parametrize("s", [1, 3, 8, 16])
def test_gram_matches_numpy(orc, s):
    rng = np.random.default_rng(7)
    X = rng.integers(-5, 6, size=(301, s)).astype(float)
    Y = rng.integers(-5, 6, size=(301, s)).astype(float)
    assert np.array_equal(orc.gram(X, Y), X.T @ Y)


@pytest.mark.parametrize("kind,q", KINDS)
def test_project_matches_definition(orc, kind, q):
    s = 8
    G = np.random.default_rng(1).standard_normal((s, s))
    P = orc.project(G, kind, q)
    if kind == "global":
        assert np.allclose(P, np.trace(G) / s * np.eye(s), rtol=0, atol=1e-15)
    else:
        assert np.array_equal(P, np.where(s_mask(s, kind, q), G, 0.0))


@pytest.mark.parametrize("kind,q", KINDS)
def test_bdot_axioms(orc, kind, q):
    """S-linearity, symmetry, normality, definiteness of <.,.>_S."""
    s, n = 8, 50
    rng = np.random.default_rng(11)
    X, Y, Z = (rng.standard_normal((n, s)) for _ in range(3))
    gam = random_in_S(rng, s, kind, q)
    lhs = orc.bdot(X + Y, Z @ gam, kind, q)
    rhs = orc.bdot(X, Z, kind, q) @ gam + orc.bdot(Y, Z, kind, q) @ gam
    assert np.allclose(lhs, rhs, atol=1e-12)
    assert np.allclose(orc.bdot(X, Y, kind, q), orc.bdot(Y, X, kind, q).T, atol=1e-13)
    assert np.isclose(np.trace(orc.bdot(X, Y, kind, q)), np.sum(X * Y), atol=1e-12)
    G = orc.bdot(X, X, kind, q)
    assert np.all(np.linalg.eigvalsh(G) > 0)
    assert np.all(orc.bdot(np.zeros((n, s)), np.zeros((n, s)), kind, q) == 0)
    # values stay inside the subalgebra
    if kind != "global":
        assert np.all(G[~s_mask(s, kind, q)] == 0)


# ------------------------------------------------------ Householder QR ----
@pytest.mark.parametrize("m,c", [(1, 1), (5, 5), (40, 8), (257, 32), (1000, 3)])
def test_qr_matches_lapack(orc, m, c):
    X = np.random.default_rng(m * 31 + c).standard_normal((m, c))
    Q, R = orc.householder_qr(X)
    Ql, Rl = np.linalg.qr(X)
    d = np.sign(np.diag(Rl))
    d[d == 0] = 1
    Ql, Rl = Ql * d, Rl * d[:, None]
    assert np.allclose(Q, Ql, atol=1e-12) and np.allclose(R, Rl, atol=1e-12)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert np.allclose(Q.T @ Q, np.eye(c), atol=1e-13)
    assert np.allclose(Q @ R, X, atol=1e-13 * max(1, np.abs(X).max()) * m ** 0.5)
    # R^T R is the Cholesky factorisation of the Gram matrix
    Lc = np.linalg.cholesky(X.T @ X)
    assert np.allclose(R, Lc.T, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("case", ["zero_col", "dup_col", "zero_all", "neg_diag_only"])
def test_qr_rank_deficient(orc, case):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((30, 6))
    if case == "zero_col":
        X[:, 2] = 0
    elif case == "dup_col":
        X[:, 4] = X[:, 1]
    elif case == "zero_all":
        X[:] = 0
    else:
        X = np.zeros((30, 6))
        X[0, 0] = -3.0
    Q, R = orc.householder_qr(X)
    assert np.allclose(Q.T @ Q, np.eye(6), atol=1e-13)   # still orthonormal (artificial directions)
    assert np.allclose(Q @ R, X, atol=1e-13)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)


@pytest.mark.parametrize("kind,q", KINDS)
def test_normalizer_definition(orc, kind, q):
    """X = Y N, <Y,Y>_S = I, N in S (upper triangular per S-block)."""
    s, n = 8, 64
    X = np.random.default_rng(2).standard_normal((n, s))
    Y, N = orc.normalize(X, kind, q)
    assert np.allclose(Y @ N, X, atol=1e-13)
    assert np.allclose(orc.bdot(Y, Y, kind, q), np.eye(s), atol=1e-13)
    if kind != "global":
        assert np.all(N[~s_mask(s, kind, q)] == 0)
    else:
        assert np.allclose(N, N[0, 0] * np.eye(s))
    assert np.allclose(np.tril(N, -1), 0) and np.all(np.diag(N) >= 0)


@pytest.mark.parametrize("kind,q", KINDS)
def test_normalizer_rank_deficient(orc, kind, q):
    s, n = 8, 40
    X = np.random.default_rng(9).standard_normal((n, s))
    X[:, 3] = 0.0
    X[:, 6] = X[:, 1]
    Y, N = orc.normalize(X, kind, q)
    assert np.allclose(Y @ N, X, atol=1e-13)
    assert np.allclose(orc.bdot(Y, Y, kind, q), np.eye(s), atol=1e-13)
    Y0, N0 = orc.normalize(np.zeros((n, s)), kind, q)
    assert np.all(N0 == 0) and np.allclose(orc.bdot(Y0, Y0, kind, q), np.eye(s))


def test_normalizer_parallel_closed_form(orc):
    X = np.random.default_rng(4).standard_normal((20, 5))
    Y, N = orc.normalize(X, "parallel")
    nrm = np.linalg.norm(X, axis=0)
    assert np.allclose(np.diag(N), nrm) and np.allclose(Y, X / nrm)


def test_normalizer_global_closed_form(orc):
    X = np.random.default_rng(4).standard_normal((20, 5))
    Y, N = orc.normalize(X, "global")
    c = np.linalg.norm(X) / np.sqrt(5)
    assert np.allclose(N, c * np.eye(5)) and np.allclose(Y, X / c)


# --------------------------------------------------- small algebra in S ----
@pytest.mark.parametrize("kind,q", KINDS)
def test_chol_solve(orc, kind, q):
    s = 8
    rng = np.random.default_rng(3)
    M = rng.standard_normal((40, s))
    A = orc.project(M.T @ M, kind, q)
    B = orc.project(rng.standard_normal((s, s)), kind, q) if kind != "global" else 2.5 * np.eye(s)
    st, X = orc.chol_solve(A, B, kind, q)
    assert st == 0
    assert np.allclose(X, np.linalg.solve(A, B), atol=1e-12)
    st, _ = orc.chol_solve(-A, B, kind, q)
    assert st == orc.E_BREAKDOWN


def test_eigenvalues_and_kappa(orc):
    rng = np.random.default_rng(8)
    for s in (1, 2, 5, 8, 16, 32):
        M = rng.standard_normal((60, s))
        A = M.T @ M
        assert np.allclose(np.sort(orc.sym_eigenvalues(A)), np.linalg.eigvalsh(A), rtol=1e-12, atol=1e-12)
        d = np.sqrt(np.diag(A))
        ev = np.linalg.eigvalsh(A / d[:, None] / d[None, :])
        assert np.isclose(orc.kappa_D(A), ev[-1] / ev[0], rtol=1e-10)
    D = np.diag(rng.uniform(1, 1e6, 8))
    assert orc.kappa_D(D) == 1.0                     # equals 1 for diagonal matrices
    assert orc.kappa_D(-np.eye(3)) == np.inf


def test_reortho_test_reading(orc):
    eps = orc.eps_f64()
    assert not orc.reortho_fires(0.0, 1e300, eps)
    assert orc.reortho_fires(np.inf, 1.0, eps)
    thr = 1.0 / (1e3 * np.sqrt(eps))                # ~6.7e4 for eta = 1000 in double
    assert orc.reortho_fires(1e3, thr * 1.01, eps) and not orc.reortho_fires(1e3, thr * 0.99, eps)
    assert np.isclose(1.0 / (1e3 * np.sqrt(orc.eps_f32())), 2.9, rtol=0.01)


# --------------------------------------------------------- SDDMM / A^T ----
@pytest.mark.parametrize("s", [1, 4, 32])
def test_sddmm_matches_dense(orc, s):
    A = W.random_csr(60, 60, 0.15, seed=s, integer=True, empty_rows=(5,))
    rng = np.random.default_rng(s)
    L = rng.integers(-3, 4, size=(60, s)).astype(float)
    X = rng.integers(-3, 4, size=(60, s)).astype(float)
    dense = -(L @ X.T)
    rows = np.repeat(np.arange(60), np.diff(A.rowptr))
    assert np.array_equal(orc.sddmm(A, L, X, -1.0), dense[rows, A.colind])


def test_csr_transpose_matches_scipy(orc):
    A = W.random_csr(120, 120, 0.05, seed=3, integer=False, empty_rows=(0, 7))
    rpT, ciT, vT, perm = orc.csr_transpose(A)
    S = scipy.sparse.csr_matrix((A.val, A.colind, A.rowptr), shape=(A.n, A.n)).T.tocsr()
    S.sort_indices()
    assert np.array_equal(rpT, S.indptr) and np.array_equal(ciT, S.indices)
    assert np.array_equal(vT, S.data) and np.array_equal(vT, A.val[perm])
