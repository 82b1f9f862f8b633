"""GPU parity of the block CG solver (bkry_cg_solve) against the oracle.

Solutions are compared at equal iteration counts (tol = 0, same maxit): both
sides then run the same arithmetic and must agree to a relative error of
1e-10 in FP64.  Converged solves are compared on iteration counts, residual
histories and the FP64 true residual.  eta is pinned at 0 and infinity, and
at intermediate values whose kappa_D decisions are clear of the threshold
(a kappa_D within rounding of the threshold can go either way)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, h, rel, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")

SUBS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]


def gpu_cg(h, A, B, X0=None, **kw):
    X, info = P.bkry_cg_solve(h, dev_csr(P, A), to_dev(B), None if X0 is None else to_dev(X0), **kw)
    return to_np(X), info


@pytest.mark.parametrize("kind,q", SUBS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_cg_poisson32_full_solve(orc, h, kind, q, eta):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("cg poisson32", kind, eta)
    X, info = gpu_cg(h, A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    ro = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    assert info["converged"] and ro["converged"]
    assert abs(info["iters"] - ro["iters"]) <= 1
    assert info["reorth"] - ro["reorth"] in (0, info["iters"] - ro["iters"])
    k = min(len(info["hist"]), len(ro["hist"]))
    assert np.allclose(info["hist"][:k], ro["hist"][:k], rtol=1e-7, atol=1e-15)
    assert max(info["true_relres"]) <= 1e-10 * 1.5
    # equal iteration counts: identical arithmetic up to rounding
    r2 = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=info["iters"], eta=eta)
    assert rel(X, r2["X"]) < 1e-10


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("kind,q", [("block", 1), ("parallel", 1), ("hybrid", 2), ("bglobal", 2)])
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_cg_widths_fixed_iterations(orc, h, s, kind, q, eta):
    if kind in ("hybrid", "bglobal") and s % q:
        pytest.skip("q must divide s")
    A = W.laplace_2d(41)                    # n = 1681: several tiles and a ragged tail
    B = W.uniform_block(A.n, s, s)
    X0 = 0.01 * W.gaussian_block(A.n, s, 100 + s)
    for k in (1, 7):
        say("cg widths", s, kind, eta, k)
        X, info = gpu_cg(h, A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        ro = orc.bcg(A, B, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        assert info["iters"] == ro["iters"] == k and info["status"] == P.NOT_CONVERGED
        assert rel(X, ro["X"]) < 1e-10


@pytest.mark.parametrize("kind,q", SUBS)
def test_cg_eta_1e4_converges(orc, h, kind, q):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("cg eta 1e4", kind)
    X, info = gpu_cg(h, A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=1e4)
    assert info["converged"] and max(info["true_relres"]) <= 1.5e-10
    Xs = np.linalg.solve(A.to_dense(), B)
    assert rel(X, Xs) < 1e-7


ETAS = [1e2, 1e3, 1e4, 1e5, 1e6, 1e7]


@pytest.mark.parametrize("name,s,kind,q", [("poisson32", 4, "block", 1), ("laplace41", 8, "block", 1),
                                           ("laplace41", 16, "block", 1), ("laplace41", 16, "hybrid", 2),
                                           ("laplace41", 32, "block", 1)])
def test_cg_reortho_decisions_match_oracle(orc, h, name, s, kind, q):
    """Intermediate eta: the kappa_D test fires at the same iterations as
    the oracle's (same iteration and re-orthonormalisation counts, same
    residual history).  Each eta is used only where every kappa_D of the
    oracle's run is at least 1e-6 (relative) away from the threshold
    1 / (eta sqrt(eps)), so that rounding cannot decide.  Histories agree
    to 1e-6 relative or 1e-13 absolute: perturbing B by one ulp moves the
    oracle's own s = 32 history by up to 2e-14 in its last steps."""
    if name == "poisson32":
        A, B, _ = W.build_workload("poisson2d_32x32_s4")
    else:
        A = W.laplace_2d(41)
        B = W.uniform_block(A.n, s, s)
    sq = np.sqrt(orc.eps_f64())
    used = 0
    for eta in ETAS:
        ro = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=3000, eta=eta, hist_cap=3000, record_blocks=3000)
        kd = [orc.kappa_D(orc.bdot(Pk, orc.spmm(A, Pk), kind, q)) for Pk in ro["Pk"]]
        if min(abs(eta * k * sq - 1.0) for k in kd) < 1e-6:
            continue
        used += 1
        say("cg reortho decisions", name, s, kind, eta)
        X, info = gpu_cg(h, A, B, kind=kind, q=q, tol=1e-10, maxit=3000, eta=eta, hist_cap=3000)
        assert info["converged"] and ro["converged"]
        assert (info["iters"], info["reorth"]) == (ro["iters"], ro["reorth"])
        assert np.allclose(info["hist"], ro["hist"], rtol=1e-6, atol=1e-13)
    assert used >= 4


def test_cg_edge_cases(orc, h):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("cg edges: zero rhs")
    X, info = gpu_cg(h, A, np.zeros_like(B), tol=1e-10)
    assert info["converged"] and info["iters"] == 0 and np.all(X == 0)
    say("cg edges: zero column, eta 0 -> breakdown")
    Bz = B.copy()
    Bz[:, 2] = 0.0
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, A, Bz, eta=0.0, tol=1e-10)
    assert e.value.code == P.E_BREAKDOWN
    say("cg edges: zero column, eta inf")
    X, info = gpu_cg(h, A, Bz, eta=np.inf, tol=1e-10, maxit=2000)
    assert info["converged"] and np.abs(X[:, 2]).max() < 1e-12
    say("cg edges: non-SPD")
    negA = W.Csr(A.n, A.rowptr, A.colind, -A.val)
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, negA, B, eta=0.0)
    assert e.value.code == P.E_BREAKDOWN
    say("cg edges: maxit 1 and 0")
    X, info = gpu_cg(h, A, B, tol=1e-10, maxit=1)
    assert info["status"] == P.NOT_CONVERGED and info["iters"] == 1
    X, info = gpu_cg(h, A, B, tol=1e-10, maxit=0)
    assert info["iters"] == 0 and np.all(X == 0)
    say("cg edges: invalid q / p")
    with pytest.raises(P.BkryError):
        gpu_cg(h, A, B, kind="hybrid", q=3)
    with pytest.raises(P.BkryError):
        gpu_cg(h, A, np.zeros((A.n, 33)))
    say("cg edges: nan rhs")
    Bn = B.copy()
    Bn[5, 1] = np.nan
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, A, Bn, eta=0.0, tol=1e-10)
    assert e.value.code == P.E_NONFINITE


@pytest.mark.parametrize("s", [16, 32])
def test_cg_edge_cases_wide(h, s):
    """The wide blocks' coefficient steps run in launches of their own (the
    alpha step as two workgroups side by side): their failures must be
    reported as in the fused form."""
    A = W.laplace_2d(32)
    B = W.uniform_block(A.n, s, 7)
    say("cg wide edges: zero column, eta 0 -> breakdown", s)
    Bz = B.copy()
    Bz[:, 3] = 0.0
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, A, Bz, eta=0.0, tol=1e-10)
    assert e.value.code == P.E_BREAKDOWN
    say("cg wide edges: zero column, eta inf", s)
    X, info = gpu_cg(h, A, Bz, eta=np.inf, tol=1e-10, maxit=2000)
    assert info["converged"] and np.abs(X[:, 3]).max() < 1e-12
    say("cg wide edges: non-SPD", s)
    negA = W.Csr(A.n, A.rowptr, A.colind, -A.val)
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, negA, B, eta=0.0)
    assert e.value.code == P.E_BREAKDOWN
    say("cg wide edges: nan rhs", s)
    Bn = B.copy()
    Bn[5, 1] = np.nan
    with pytest.raises(P.BkryError) as e:
        gpu_cg(h, A, Bn, eta=0.0, tol=1e-10)
    assert e.value.code == P.E_NONFINITE
    say("cg wide edges: eta 1e4 full solve", s)
    X, info = gpu_cg(h, A, B, eta=1e4, tol=1e-10, maxit=2000)
    assert info["converged"] and max(info["true_relres"]) <= 1.5e-10
    assert rel(X, np.linalg.solve(A.to_dense(), B)) < 1e-8


def test_cg_deterministic(h):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("cg determinism")
    X1, i1 = gpu_cg(h, A, B, tol=1e-10, eta=1e4)
    X2, i2 = gpu_cg(h, A, B, tol=1e-10, eta=1e4)
    assert np.array_equal(X1, X2) and i1["iters"] == i2["iters"]


def test_cg_exhausted_krylov_space(orc, h):
    """Rank-deficient residual when the block Krylov space is exhausted:
    without re-orthonormalisation (eta = 0) alpha is singular up to rounding,
    so what happens next depends on the rounding of its last pivot: a
    non-positive pivot stops the solve (the oracle's case), a positive one of
    rounding size lets it go on.  Either way the outcome must be reported
    honestly: an error code, or a result whose convergence flag agrees with
    the FP64 true residual.  With eta = inf it converges (same as the
    oracle)."""
    A = W.laplace_2d(7)
    B = W.uniform_block(A.n, 4, 4)
    say("cg exhausted")
    try:
        X, info = gpu_cg(h, A, B, eta=0.0, tol=1e-12, maxit=500)
        if info["converged"]:
            assert max(info["true_relres"]) <= 1e-10
            assert rel(X, np.linalg.solve(A.to_dense(), B)) < 1e-8
    except P.BkryError as e:
        assert e.code in (P.E_BREAKDOWN, P.E_NONFINITE)
    X, info = gpu_cg(h, A, B, eta=np.inf, tol=1e-12, maxit=500)
    assert info["converged"] and rel(X, np.linalg.solve(A.to_dense(), B)) < 1e-10


@pytest.mark.parametrize("kind,q", [("block", 1), ("hybrid", 2)])
def test_cg_laplace128_full_size_fixed_iterations(orc, h, kind, q):
    """The 128^3 / p = 8 workload at its full size, 3 iterations, eta = inf."""
    A, B, _ = W.build_workload("laplace3d_128_s8")
    say("cg 128^3 fixed", kind)
    X, info = gpu_cg(h, A, B, kind=kind, q=q, tol=0.0, maxit=3, eta=np.inf)
    ro = orc.bcg(A, B, kind=kind, q=q, tol=0.0, maxit=3, eta=np.inf)
    assert rel(X, ro["X"]) < 1e-10


def test_cg_laplace128_time_to_tol(h):
    """Full solve at full size: the FP64 true residual meets 1e-10 (property
    check at a size the oracle cannot repeat quickly)."""
    A, B, _ = W.build_workload("laplace3d_128_s8")
    say("cg 128^3 solve")
    X, info = gpu_cg(h, A, B, kind="block", tol=1e-10, maxit=3000, eta=1e4)
    assert info["converged"]
    assert max(info["true_relres"]) <= 2e-10
    say("cg 128^3 iters", info["iters"], "reorth", info["reorth"], "s", info["seconds"])
