"""Pins for the oracle adjoint of the block solve A X = B.

For L(X) with gradient G = dL/dX at X = A^-1 B, the adjoint is
Lambda = A^-T G, dL/dB = Lambda and dL/dA = -Lambda X^T, restricted to the
pattern of A for dL/dval.  Checked against dense LU and against central finite
differences of the loss L = 1/2 |X - T|_F^2.
"""
import numpy as np
import pytest

import workloads as W


def test_adjoint_matches_dense_lu(orc):
    A = W.diffusion_7pt_var(4, seed=11)
    D = A.to_dense()
    B = W.gaussian_block(A.n, 3, 1)
    T = W.gaussian_block(A.n, 3, 2)
    X = np.linalg.solve(D, B)
    G = X - T
    lam_ref = np.linalg.solve(D.T, G)
    dA = -lam_ref @ X.T
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    lam, dval, r = orc.adjoint(A, X, G, tol=1e-14)
    assert r["converged"]
    assert np.allclose(lam, lam_ref, atol=1e-11 * np.abs(lam_ref).max())
    assert np.allclose(dval, dA[rows, A.colind], atol=1e-11 * np.abs(dA).max())


def test_adjoint_nonsymmetric_uses_transpose(orc):
    A = W.convdiff_2d(5, pe_h=1.0)
    D = A.to_dense()
    rpT, ciT, vT, _ = orc.csr_transpose(A)
    AT = W.Csr(A.n, rpT, ciT, vT)
    assert np.array_equal(AT.to_dense(), D.T)
    B = W.gaussian_block(A.n, 2, 3)
    X = np.linalg.solve(D, B)
    G = np.ones_like(X)
    # block CG needs SPD; check the SDDMM part with the exact Lambda instead
    lam = np.linalg.solve(D.T, G)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.allclose(orc.sddmm(A, lam, X, -1.0), (-lam @ X.T)[rows, A.colind], atol=1e-12)


def test_adjoint_central_finite_differences(orc):
    """Perturb a symmetric pair (a_ij, a_ji) by +-h; the derivative of the loss
    is g_ij + g_ji (for i != j) and g_ii on the diagonal."""
    A = W.diffusion_7pt_var(3, seed=13)
    D = A.to_dense()
    B = W.gaussian_block(A.n, 2, 4)
    T = W.gaussian_block(A.n, 2, 5)
    X = np.linalg.solve(D, B)
    lam, dval, _ = orc.adjoint(A, X, X - T, tol=1e-14)
    g = np.zeros_like(D)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    g[rows, A.colind] = dval
    rng = np.random.default_rng(5005)
    h = 1e-6
    for k in rng.choice(A.nnz, 12, replace=False):
        i, j = rows[k], A.colind[k]
        E = np.zeros_like(D)
        E[i, j] = 1.0
        E[j, i] = 1.0
        Xp = np.linalg.solve(D + h * E, B)
        Xm = np.linalg.solve(D - h * E, B)
        fd = 0.5 * np.sum((Xp - Xm) * (Xp + Xm - 2 * T)) / (2 * h)
        adj = g[i, j] + (g[j, i] if i != j else 0.0)
        assert abs(fd - adj) <= 1e-6 * max(1.0, abs(adj)), (i, j, fd, adj)
    # dL/dB = Lambda
    Eb = np.zeros_like(B)
    Eb[3, 1] = 1.0
    fd = (0.5 * np.sum((np.linalg.solve(D, B + h * Eb) - T) ** 2)
          - 0.5 * np.sum((np.linalg.solve(D, B - h * Eb) - T) ** 2)) / (2 * h)
    assert abs(fd - lam[3, 1]) < 1e-6 * max(1, abs(lam[3, 1]))
