"""Independent reference constructions used to pin the oracle's solvers.

None of these follow the block algorithms: they are textbook scalar CG and
brute-force minimisers over an explicitly assembled block Krylov space
(Definition "Block Krylov subspace", Ch. 3), solved with numpy least squares.
"""
import numpy as np


def subalgebra_basis(s, kind, q=1):
    """A basis of the *-subalgebra as s x s unit matrices (Definitions of
    S_G, S_P, S_B and S_BP in Ch. 3)."""
    if kind == "global":
        return [np.eye(s)]
    if kind == "parallel":
        return [np.diag(np.eye(s)[i]) for i in range(s)]
    if kind == "bglobal":
        g = s // q
        out = []
        for a in range(g):
            for b in range(g):
                E = np.zeros((g, g))
                E[a, b] = 1.0
                out.append(np.kron(np.eye(q), E))
        return out
    g = s if kind == "block" else s // q
    out = []
    for a in range(s):
        for b in range(s):
            if a // g == b // g:
                E = np.zeros((s, s))
                E[a, b] = 1.0
                out.append(E)
    return out


def krylov_basis(A, R0, k, kind, q=1):
    """Columns vec(A^i R0 E) for i < k and E in the subalgebra basis, as an
    orthonormal basis (QR with rank truncation) of the block Krylov space."""
    n, s = R0.shape
    cols = []
    Ai = R0.copy()
    for _ in range(k):
        for E in subalgebra_basis(s, kind, q):
            cols.append((Ai @ E).reshape(-1, order="F"))
        Ai = A @ Ai
    K = np.array(cols).T
    U, sv, _ = np.linalg.svd(K, full_matrices=False)
    r = int(np.sum(sv > sv[0] * 1e-12))
    return U[:, :r]


def galerkin_minimiser(A, B, X0, k, kind, q=1):
    """argmin over X0 + K_k^S(A, R0) of |X - X*|_{A,F} (energy minimisation
    characterising the k-th block CG iterate)."""
    n, s = B.shape
    R0 = B - A @ X0
    U = krylov_basis(A, R0, k, kind, q)
    Ahat = np.kron(np.eye(s), A)
    c = np.linalg.solve(U.T @ Ahat @ U, U.T @ R0.reshape(-1, order="F"))
    return X0 + (U @ c).reshape((n, s), order="F")


def galerkin_minimiser_prec(A, B, X0, k, kind, q, minv):
    """argmin over X0 + K_k^S(M^-1 A, M^-1 R0) of |X - X*|_{A,F} for the
    diagonal preconditioner M^-1 = diag(minv): the k-th preconditioned block
    CG iterate (the minimisation property of Ch. 4 with M != I)."""
    n, s = B.shape
    R0 = B - A @ X0
    Mi = np.diag(minv)
    U = krylov_basis(Mi @ A, Mi @ R0, k, kind, q)
    Ahat = np.kron(np.eye(s), A)
    c = np.linalg.solve(U.T @ Ahat @ U, U.T @ R0.reshape(-1, order="F"))
    return X0 + (U @ c).reshape((n, s), order="F")


def galerkin_minimiser_precmat(A, B, X0, k, kind, q, Minv):
    """As galerkin_minimiser_prec for a dense M^-1 (any SPD preconditioner)."""
    n, s = B.shape
    R0 = B - A @ X0
    U = krylov_basis(Minv @ A, Minv @ R0, k, kind, q)
    Ahat = np.kron(np.eye(s), A)
    c = np.linalg.solve(U.T @ Ahat @ U, U.T @ R0.reshape(-1, order="F"))
    return X0 + (U @ c).reshape((n, s), order="F")


def ssor_matrix(A, colors, omega):
    """The multicolour SSOR matrix written out from its definition: with the
    rows ordered by colour, A = L + D + U (L: columns of smaller colour),
    M = (D + omega L) D^-1 (D + omega U) / (omega (2 - omega))."""
    d = np.diag(A).copy()
    lower = colors[None, :] < colors[:, None]
    upper = colors[None, :] > colors[:, None]
    L = np.where(lower, A, 0.0)
    U = np.where(upper, A, 0.0)
    D = np.diag(d)
    return (D + omega * L) @ np.diag(1.0 / d) @ (D + omega * U) / (omega * (2.0 - omega))


def residual_minimiser(A, B, X0, k, kind, q=1):
    """argmin over X0 + K_k^S(A, R0) of |B - A X|_F (the block GMRes iterate)."""
    n, s = B.shape
    R0 = B - A @ X0
    U = krylov_basis(A, R0, k, kind, q)
    Ahat = np.kron(np.eye(s), A)
    c, *_ = np.linalg.lstsq(Ahat @ U, R0.reshape(-1, order="F"), rcond=None)
    return X0 + (U @ c).reshape((n, s), order="F")


def textbook_cg(A, b, x0, k):
    """k steps of the scalar conjugate gradient method (Hestenes-Stiefel)."""
    x = x0.astype(float).copy()
    r = b - A @ x
    p = r.copy()
    rr = r @ r
    for _ in range(k):
        q = A @ p
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def energy_fro(A, E):
    return float(np.sqrt(np.sum(E * (A @ E))))


def laplace2d_eigpair(N, i, j):
    """Closed-form eigenpair of the N x N Dirichlet 5-point Laplacian
    [-1; -1 4 -1; -1] (x fastest ordering)."""
    h = 1.0 / (N + 1)
    x = np.arange(1, N + 1) * h
    u = np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).reshape(-1)  # [y][x]
    lam = 4.0 - 2.0 * np.cos(i * np.pi * h) - 2.0 * np.cos(j * np.pi * h)
    return lam, u


def laplace2d_extremes(N):
    h = 1.0 / (N + 1)
    return 4.0 - 4.0 * np.cos(np.pi * h), 4.0 + 4.0 * np.cos(np.pi * h)
