"""Differentiable block solve (paper_2104_02494_amd.block_solve): gradients
from the adjoint solve and the sampled product on the pattern, against the
oracle's adjoint and central finite differences.

Finite differences follow the symmetric-pair protocol: a single off-diagonal
value cannot be perturbed alone (A would stop being symmetric and CG would
not apply), so a_ij and a_ji move together and the difference quotient is
compared with g_ij + g_ji (g_ii for a diagonal entry).  The loss difference
is formed as 1/2 <X+ - X-, X+ + X- - 2T>, which avoids the cancellation of
L(+h) - L(-h) for a loss of order n * p.

Step h = 1e-4: the two perturbed solves stop after their own iteration
counts (tol 1e-13), so their solution errors do not cancel and enter the
quotient as ~ tol * kappa / h, while the central-difference truncation error
is O(h^2).  At h = 1e-6 the first term reached 3e-5 of |g| on the 64^3
workload; at h = 1e-4 both terms stay below 1e-6 there."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, h, rel, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")
torch = pytest.importorskip("torch")


def grads(h, A, B, T, tol=1e-13):
    Ad = dev_csr(P, A)
    vals = Ad.val.clone().requires_grad_(True)
    Bd = to_dev(B).requires_grad_(True)
    X = P.block_solve(vals, Bd, Ad, h, tol=tol, eta=np.inf)
    loss = 0.5 * ((X - to_dev(T)) ** 2).sum()
    loss.backward()
    return to_np(X.detach()), to_np(vals.grad), to_np(Bd.grad)


def test_adjoint_vs_oracle(orc, h):
    A = W.diffusion_7pt_var(8, seed=1005)        # n = 512
    B = W.gaussian_block(A.n, 4, 2005)
    T = W.gaussian_block(A.n, 4, 3005)
    say("adjoint vs oracle")
    X, dv, dB = grads(h, A, B, T)
    ro = orc.bcg(A, B, tol=1e-13, maxit=5000, eta=np.inf)
    lam, dv_or, _ = orc.adjoint(A, ro["X"], ro["X"] - T, eta=np.inf)
    assert rel(X, ro["X"]) < 1e-10
    assert rel(dB, lam) < 1e-9
    assert rel(dv, dv_or) < 1e-9


def test_adjoint_vs_oracle_wide(orc, h):
    """The 32 right-hand sides of the 64^3 workload on a 16^3 instance of its
    generator (n = 4,096): solution, dL/dB and dL/dvalues against the
    oracle's adjoint (oracle block CG on A^T, then the sampled product)."""
    A = W.diffusion_7pt_var(16, seed=1005)
    B = W.gaussian_block(A.n, 32, 2005)
    T = W.gaussian_block(A.n, 32, 3005)
    say("adjoint vs oracle p=32 16^3")
    X, dv, dB = grads(h, A, B, T)
    ro = orc.bcg(A, B, tol=1e-13, maxit=5000, eta=np.inf)
    lam, dv_or, _ = orc.adjoint(A, ro["X"], ro["X"] - T, eta=np.inf)
    assert rel(X, ro["X"]) < 1e-10
    assert rel(dB, lam) < 1e-9
    assert rel(dv, dv_or) < 1e-9


def pair_index(A):
    """k -> position of the transposed entry (j, i) of entry k = (i, j)."""
    pos = {}
    for i in range(A.n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            pos[(i, int(A.colind[k]))] = k
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    return np.array([pos[(int(A.colind[k]), int(rows[k]))] for k in range(A.nnz)]), rows


def fd_check(h, A, B, T, entries, hstep=1e-4):
    _, dv, _ = grads(h, A, B, T)
    tr, rows = pair_index(A)
    Ad = dev_csr(P, A)
    Bd = to_dev(B)
    worst = 0.0
    for k in entries:
        kt = tr[k]
        vp = A.val.copy()
        vm = A.val.copy()
        vp[k] += hstep
        vm[k] -= hstep
        if kt != k:
            vp[kt] += hstep
            vm[kt] -= hstep
        Xp, _ = P.bkry_cg_solve(h, P.CsrMatrix(Ad.n, Ad.rowptr, Ad.colind, to_dev(vp)), Bd, tol=1e-13,
                                maxit=20000, eta=np.inf)
        Xm, _ = P.bkry_cg_solve(h, P.CsrMatrix(Ad.n, Ad.rowptr, Ad.colind, to_dev(vm)), Bd, tol=1e-13,
                                maxit=20000, eta=np.inf)
        Xp, Xm = to_np(Xp), to_np(Xm)
        fd = 0.5 * np.sum((Xp - Xm) * (Xp + Xm - 2 * T)) / (2 * hstep)
        adj = dv[k] + (dv[kt] if kt != k else 0.0)
        err = abs(fd - adj) / max(1.0, abs(adj))
        worst = max(worst, err)
    return worst


def test_adjoint_finite_differences(h):
    """64 pattern entries sampled uniformly (seed 5005) on a 16^3 grid."""
    A = W.diffusion_7pt_var(16, seed=1005)       # n = 4096
    B = W.gaussian_block(A.n, 8, 2005)
    T = W.gaussian_block(A.n, 8, 3005)
    entries = np.random.default_rng(5005).choice(A.nnz, size=64, replace=False)
    say("adjoint FD 16^3")
    assert fd_check(h, A, B, T, entries) <= 1e-5


def test_adjoint_full_size_finite_differences(h):
    """The 64^3 / p = 32 workload itself, 64 pattern entries sampled
    uniformly (seed 5005), two perturbed solves each."""
    A, B, extra = W.build_workload("diffusion7var_64_s32")
    T = extra["target"]
    entries = np.random.default_rng(5005).choice(A.nnz, size=64, replace=False)
    say("adjoint FD 64^3")
    assert fd_check(h, A, B, T, entries) <= 1e-5
