"""GPU parity of restarted block GMRes (bkry_gmres_solve) against the oracle.

The GPU orthogonalises with classical Gram-Schmidt applied twice, the oracle
with modified Gram-Schmidt; in exact arithmetic both give the same Arnoldi
basis, and on these well-conditioned problems the iterates agree to a
relative error of 1e-10 at equal step counts.  Converged solves are compared
on the FP64 true residual."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, h, rel, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")

SUBS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]
# widths: 4, the 8 of the 1024^2 convection-diffusion workload, and the wide
# blocks whose CGS2 block combinations and Givens steps take other code paths
WIDTHS = [4, 8, 16, 32]


def gpu_gm(h, A, B, **kw):
    X, info = P.bkry_gmres_solve(h, dev_csr(P, A), to_dev(B), **kw)
    return to_np(X), info


def fixed_problem(p):
    # the block Krylov space after the longest case (17 steps) stays well
    # inside the space: 17 p < n
    A = W.convdiff_2d(24 if p <= 8 else 40)     # nonsymmetric, n = 576 or 1600
    return A, W.gaussian_block(A.n, p, 7 + p)


@pytest.mark.parametrize("p", WIDTHS)
@pytest.mark.parametrize("kind,q", SUBS)
@pytest.mark.parametrize("steps,restart", [(1, 30), (6, 30), (17, 30), (23, 5)])
def test_gmres_fixed_steps(orc, h, p, kind, q, steps, restart):
    A, B = fixed_problem(p)
    say("gmres fixed", p, kind, steps, restart)
    X, info = gpu_gm(h, A, B, kind=kind, q=q, tol=0.0, maxit=steps, restart=restart)
    ro = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=steps, restart=restart)
    assert info["iters"] == ro["iters"] == steps
    assert info["outer_iters"] == ro["cycles"]
    assert rel(X, ro["X"]) < 1e-10


@pytest.mark.parametrize("p", WIDTHS)
@pytest.mark.parametrize("kind,q", SUBS)
def test_gmres_converges_like_oracle(orc, h, p, kind, q):
    A = W.convdiff_2d(32)
    B = W.gaussian_block(A.n, p, 8 + p)
    say("gmres solve", p, kind)
    X, info = gpu_gm(h, A, B, kind=kind, q=q, tol=1e-10, maxit=3000, restart=30, hist_cap=3000)
    ro = orc.bgmres(A, B, kind=kind, q=q, tol=1e-10, maxit=3000, restart=30, hist_cap=3000)
    assert info["converged"] and ro["converged"]
    assert abs(info["iters"] - ro["iters"]) <= 1
    assert max(info["true_relres"]) <= 1e-9
    k = min(len(info["hist"]), len(ro["hist"])) - 1
    hg, ho = np.asarray(info["hist"][:k]), np.asarray(ro["hist"][:k])
    # relative agreement while the residual is large; near the tolerance the
    # two orthogonalisations (CGS2 here, MGS in the oracle) differ by their
    # rounding: MGS loses orthogonality in proportion to |R0| / |R_k|, so the
    # histories differ by an absolute amount of about eps kappa(A) k sqrt(k p)
    # (in units of |R0|; measured up to 2.4e-11 at p = 32, where 30 steps
    # span 960 of the 1024 dimensions).  Half the stopping tolerance bounds
    # it and keeps the stopping steps within one of each other.
    diff = np.abs(hg - ho)
    say("gmres hist worst rel", float((diff / ho).max()), "worst abs", float(diff.max()))
    assert np.all(diff <= 1e-6 * ho + 5e-11)


def test_gmres_edge_cases(orc, h):
    A = W.convdiff_2d(16)
    B = W.gaussian_block(A.n, 4, 9)
    say("gmres zero rhs")
    X, info = gpu_gm(h, A, np.zeros_like(B), tol=1e-10, maxit=100)
    assert info["converged"] and info["iters"] == 0 and np.all(X == 0)
    say("gmres rank-deficient rhs")
    Bd = B.copy()
    Bd[:, 3] = Bd[:, 1]
    X, info = gpu_gm(h, A, Bd, tol=1e-10, maxit=600, restart=30)
    assert info["converged"] and max(info["true_relres"]) <= 1e-9
    assert rel(X, np.linalg.solve(A.to_dense(), Bd)) < 1e-7
    say("gmres maxit 0")
    X, info = gpu_gm(h, A, B, tol=1e-10, maxit=0)
    assert info["iters"] == 0 and np.all(X == 0) and not info["converged"]
    say("gmres invalid restart")
    with pytest.raises(P.BkryError):
        gpu_gm(h, A, B, restart=0)
    with pytest.raises(P.BkryError):
        gpu_gm(h, A, B, restart=201)


@pytest.mark.parametrize("r", [0, 2])
def test_gmres_invariant_krylov_space(h, r):
    """A with three distinct eigenvalues: the block Krylov space of 4
    right-hand sides is invariant after three steps, so the third Arnoldi
    block is zero and its CholeskyQR fails (the Householder fallback of the
    normaliser is needed inside a cycle).  The cycle must still end with the
    exact solution."""
    rng = np.random.default_rng(31)
    d = rng.choice([1.0, 2.0, 5.0], size=300)
    A = W.dense_to_csr(np.diag(d))
    B = W.gaussian_block(A.n, 4, 32)
    say("gmres invariant space", r)
    kw = dict(tol=1e-10, maxit=60, restart=30)
    if r:
        X, info = P.bkry_gmres_pipelined_solve(h, dev_csr(P, A), to_dev(B), r, **kw)
    else:
        X, info = P.bkry_gmres_solve(h, dev_csr(P, A), to_dev(B), **kw)
    X = to_np(X)
    assert info["converged"] and info["iters"] <= 4, info
    assert max(info["true_relres"]) <= 1e-9
    assert rel(X, B / d[:, None]) < 1e-9


def test_gmres_deterministic(h):
    A = W.convdiff_2d(24)
    B = W.gaussian_block(A.n, 8, 3)
    say("gmres determinism")
    X1, i1 = gpu_gm(h, A, B, tol=1e-10, maxit=500)
    X2, i2 = gpu_gm(h, A, B, tol=1e-10, maxit=500)
    assert np.array_equal(X1, X2) and i1["iters"] == i2["iters"]


def test_gmres_full_size_first_cycle_vs_oracle(orc, h):
    """The 1024^2 convection-diffusion workload with 8 right-hand sides: the
    first GMRes(30) cycle (30 Arnoldi steps from X0 = 0) against the oracle's
    modified Gram-Schmidt Arnoldi at equal step counts."""
    A, B, _ = W.build_workload("convdiff2d_1024_s8")
    say("gmres 1024^2 first cycle vs oracle")
    X, info = gpu_gm(h, A, B, kind="block", tol=0.0, maxit=30, restart=30)
    assert info["iters"] == 30 and info["outer_iters"] == 1
    ro = orc.bgmres(A, B, kind="block", tol=0.0, maxit=30, restart=30)
    assert ro["iters"] == 30
    assert rel(X, ro["X"]) < 1e-10


def test_gmres_full_size_cycle(h):
    """The 1024^2 convection-diffusion workload with 8 right-hand sides, one
    GMRes(30) cycle at full size: the implicit residual of the last step
    (from the Givens-rotated least-squares problem) must equal the FP64 true
    residual recomputed from X (property check at a size the oracle cannot
    repeat quickly)."""
    A, B, _ = W.build_workload("convdiff2d_1024_s8")
    say("gmres 1024^2 cycle")
    X, info = gpu_gm(h, A, B, kind="block", tol=0.0, maxit=30, restart=30, hist_cap=30)
    assert info["iters"] == 30 and info["outer_iters"] == 1
    implicit = info["hist"][-1]
    true = max(info["true_relres"])
    assert abs(implicit - true) <= 1e-6 * true


# ---- pipelined Gram-Schmidt (bkry_gmres_pipelined_solve) against the oracle's
# pipelined orthogonalisation with the same window ---------------------------
@pytest.mark.parametrize("r", [1, 2, 3, 30])
@pytest.mark.parametrize("p", WIDTHS)
@pytest.mark.parametrize("kind,q", SUBS)
@pytest.mark.parametrize("steps,restart", [(1, 30), (9, 30), (17, 30), (23, 5)])
def test_pipelined_gmres_fixed_steps(orc, h, r, p, kind, q, steps, restart):
    A, B = fixed_problem(p)
    say("pipelined gmres fixed", r, p, kind, steps, restart)
    X, info = gpu_gm(h, A, B, kind=kind, q=q, tol=0.0, maxit=steps, restart=restart, pipelined=r)
    ro = orc.bgmres(A, B, kind=kind, q=q, tol=0.0, maxit=steps, restart=restart, pipelined=r)
    assert info["iters"] == ro["iters"] == steps
    assert info["outer_iters"] == ro["cycles"]
    assert rel(X, ro["X"]) < 1e-10


@pytest.mark.parametrize("r", [1, 3, 29])
@pytest.mark.parametrize("p", [4, 8])
def test_pipelined_gmres_converges_like_oracle(orc, h, r, p):
    A = W.convdiff_2d(32)
    B = W.gaussian_block(A.n, p, 8 + p)
    say("pipelined gmres solve", r, p)
    X, info = gpu_gm(h, A, B, tol=1e-10, maxit=3000, restart=30, hist_cap=3000, pipelined=r)
    ro = orc.bgmres(A, B, tol=1e-10, maxit=3000, restart=30, hist_cap=3000, pipelined=r)
    assert info["converged"] and ro["converged"]
    assert abs(info["iters"] - ro["iters"]) <= 1
    assert max(info["true_relres"]) <= 1e-9
    k = min(len(info["hist"]), len(ro["hist"])) - 1
    hg, ho = np.asarray(info["hist"][:k]), np.asarray(ro["hist"][:k])
    assert np.all(np.abs(hg - ho) <= 1e-6 * ho + 5e-11)


def test_pipelined_gmres_rejects_window_zero(h):
    A = W.convdiff_2d(16)
    B = W.gaussian_block(A.n, 4, 9)
    with pytest.raises(P.BkryError):
        gpu_gm(h, A, B, pipelined=0)


def test_pipelined_gmres_full_size_cycle(h):
    """One GMRes(30) cycle with window 3 on the 1024^2 workload (p = 8): the
    implicit residual of the last step equals the FP64 true residual."""
    A, B, _ = W.build_workload("convdiff2d_1024_s8")
    say("pipelined gmres 1024^2 cycle")
    X, info = gpu_gm(h, A, B, kind="block", tol=0.0, maxit=30, restart=30, hist_cap=30, pipelined=3)
    assert info["iters"] == 30 and info["outer_iters"] == 1
    implicit = info["hist"][-1]
    true = max(info["true_relres"])
    assert abs(implicit - true) <= 1e-6 * true
