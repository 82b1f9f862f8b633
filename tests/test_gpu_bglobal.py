"""GPU checks particular to the block-global subalgebra S_BG(q) (Definition
"Relevant *-subalgebras", Ch. 3): its reductions to the block (q = 1) and
global (q = p) subalgebras run those exactly, the normaliser of a block whose
stacked groups are rank-deficient keeps its invariants, and the subalgebra
lattice G >= BG >= B shows in the iteration counts of the block CG.
Parity of BDOT, the normaliser and every solver with the oracle for
S_BG(2) and S_BG(4) is in the per-solver test files."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, h, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")


@pytest.mark.parametrize("q,same", [(1, "block"), (4, "global")])
def test_bglobal_reductions_are_exact(h, q, same):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    Ad, Bd = dev_csr(P, A), to_dev(B)
    say("bglobal q", q, "is", same)
    X1, i1 = P.bkry_cg_solve(h, Ad, Bd, kind="bglobal", q=q, tol=1e-10, maxit=2000, eta=np.inf)
    X0, i0 = P.bkry_cg_solve(h, Ad, Bd, kind=same, tol=1e-10, maxit=2000, eta=np.inf)
    assert i1["iters"] == i0["iters"] and np.array_equal(to_np(X1), to_np(X0))
    X = W.gaussian_block(5000, 4, 3)
    Xa, Xb = to_dev(X), to_dev(X)
    Na = to_np(P.bkry_tsqr(h, Xa, "bglobal", q))
    Nb = to_np(P.bkry_tsqr(h, Xb, same))
    assert np.array_equal(Na, Nb) and np.array_equal(to_np(Xa), to_np(Xb))


def test_bglobal_invalid_q(h):
    X = to_dev(W.gaussian_block(100, 6, 1))
    for q in (0, 4, 7):
        with pytest.raises(P.BkryError) as e:
            P.bkry_tsqr(h, X, "bglobal", q)
        assert e.value.code == P.E_INVALID


@pytest.mark.parametrize("case", ["shared_zero_col", "one_group_zero", "zero_all"])
def test_bglobal_normaliser_rank_deficient(orc, h, case):
    """X = Y N with <Y, Y>_BG = I and N = I (x) rho / sqrt(q), rho upper
    triangular with a non-negative diagonal; where the stacked groups keep
    full rank, Y and N are unique and must match the oracle."""
    n, s, q = 3000, 8, 2
    g = s // q
    X = W.gaussian_block(n, s, 11)
    if case == "shared_zero_col":            # column 1 of every group is zero: stacked rank g - 1
        X[:, [1, 1 + g]] = 0.0
    elif case == "one_group_zero":           # the stacked block keeps full rank
        X[:, g:] = 0.0
    else:
        X[:] = 0.0
    say("bglobal normaliser", case)
    Xd = to_dev(X)
    N = to_np(P.bkry_tsqr(h, Xd, "bglobal", q))
    Y = to_np(Xd)
    rho = N[:g, :g] * np.sqrt(q)
    for k in range(q):
        assert np.array_equal(N[k * g:(k + 1) * g, k * g:(k + 1) * g], N[:g, :g])
    assert np.all(N[orc.project(np.ones((s, s)), "bglobal", q) == 0] == 0)
    assert np.allclose(np.tril(rho, -1), 0) and np.all(np.diag(rho) >= 0)
    assert np.abs(orc.bdot(Y, Y, "bglobal", q) - np.eye(s)).max() < 1e-12
    assert np.abs(Y @ N - X).max() <= 1e-13 * max(1.0, np.abs(X).max())
    if case == "one_group_zero":
        Yo, No = orc.normalize(X, "bglobal", q)
        assert np.abs(N - No).max() < 1e-12 * np.abs(No).max()
        assert np.abs(Y - Yo).max() < 1e-11


def test_bglobal_lattice_iterations(h):
    """A larger subalgebra gives the block CG a larger search space per step
    (Ch. 3, the subalgebra lattice): iterations(global) >= iterations(BG(2))
    >= iterations(block) on the same system."""
    A = W.laplace_2d(41)
    B = W.uniform_block(A.n, 8, 5)
    Ad, Bd = dev_csr(P, A), to_dev(B)
    it = {}
    for kind, q in (("global", 1), ("bglobal", 2), ("block", 1)):
        say("bglobal lattice", kind)
        _, info = P.bkry_cg_solve(h, Ad, Bd, kind=kind, q=q, tol=1e-10, maxit=3000, eta=1e4)
        assert info["converged"] and max(info["true_relres"]) <= 1.5e-10
        it[kind] = info["iters"]
    assert it["global"] >= it["bglobal"] >= it["block"]
