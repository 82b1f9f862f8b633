"""GPU parity of the multicolour SSOR preconditioner against the oracle: the
Jones-Plassmann colouring (bkry_color) must equal the oracle's greedy
colouring in priority order bit for bit, the colour sweeps (bkry_ssor_apply)
must match the oracle's to rounding, and the SSOR-preconditioned block CG
(bkry_pcg_ssor_solve) must follow the oracle's iteration: fixed step counts
to 1e-10 relative in FP64, full solves on iteration counts, residual
histories and the FP64 true residual."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, h, rel, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")

SUBS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]
MATS = {"lap2d_41": lambda: W.laplace_2d(41), "lap3d_20": lambda: W.laplace_3d(20),
        "diff27_12": lambda: W.diffusion_27pt(12, seed=4), "var7_12": lambda: W.diffusion_7pt_var(12, seed=8),
        "randspd_3000": lambda: W.random_spd_csr(3000, 0.004, seed=5)}


def gpu_colors(h, A, prio):
    c, nc = P.bkry_color(h, dev_csr(P, A), to_dev(prio.view(np.int32)))
    return to_np(c), nc


@pytest.mark.parametrize("name", list(MATS))
def test_color_matches_oracle(orc, h, name):
    A = MATS[name]()
    prio = W.color_priorities(A.n, 21)
    prio[::5] = prio[7]                                   # ties, broken by the row index
    say("color", name)
    cg, ncg = gpu_colors(h, A, prio)
    co, nco = orc.color_greedy(A, prio)
    assert ncg == nco and np.array_equal(cg, co)


def test_color_natural_order_and_errors(orc, h):
    A = W.laplace_3d(16)
    say("color natural order")
    prio = (A.n - 1 - np.arange(A.n)).astype(np.uint32)
    c, nc = gpu_colors(h, A, prio)
    idx = np.arange(A.n)
    assert nc == 2 and np.array_equal(c, (idx % 16 + idx // 16 % 16 + idx // 256) % 2)
    say("color bad column")
    bad = W.Csr(A.n, A.rowptr, A.colind.copy(), A.val)
    bad.colind[10] = A.n + 3
    with pytest.raises(P.BkryError) as e:
        gpu_colors(h, bad, W.color_priorities(A.n, 1))
    assert e.value.code == P.E_INVALID


@pytest.mark.parametrize("s", [1, 2, 3, 4, 8, 16, 32])
@pytest.mark.parametrize("omega", [1.0, 1.4])
def test_ssor_apply_matches_oracle(orc, h, s, omega):
    A = W.diffusion_7pt_var(12, seed=8)                    # n = 1728: several tiles and a ragged tail
    prio = W.color_priorities(A.n, 3)
    cg, _ = gpu_colors(h, A, prio)
    co, _ = orc.color_greedy(A, prio)
    assert np.array_equal(cg, co)
    R = W.gaussian_block(A.n, s, 40 + s)
    say("ssor apply", s, omega)
    Z = to_np(P.bkry_ssor_apply(h, dev_csr(P, A), to_dev(cg), omega, to_dev(R)))
    st, Zo = orc.ssor_apply(A, co, omega, R)
    assert st == orc.OK
    assert np.abs(Z - Zo).max() <= 1e-12 * np.abs(Zo).max()


def test_ssor_apply_errors(orc, h):
    A = W.laplace_2d(20)
    Ad = dev_csr(P, A)
    R = to_dev(W.gaussian_block(A.n, 4, 1))
    cg, _ = gpu_colors(h, A, W.color_priorities(A.n, 2))
    say("ssor errors")
    for colors, omega in ((np.zeros(A.n, np.int32), 1.0), (cg, 2.0), (cg, 0.0),
                          (np.full(A.n, 5000, np.int32), 1.0)):
        with pytest.raises(P.BkryError) as e:
            P.bkry_ssor_apply(h, Ad, to_dev(colors), omega, R)
        assert e.value.code == P.E_INVALID
    negA = dev_csr(P, W.Csr(A.n, A.rowptr, A.colind, -A.val))
    with pytest.raises(P.BkryError) as e:
        P.bkry_ssor_apply(h, negA, to_dev(cg), 1.0, R)
    assert e.value.code == P.E_INVALID


def setup(h, orc, A, seed=17):
    prio = W.color_priorities(A.n, seed)
    cg, _ = gpu_colors(h, A, prio)
    co, _ = orc.color_greedy(A, prio)
    assert np.array_equal(cg, co)
    return to_dev(cg), co


@pytest.mark.parametrize("s", [1, 3, 4, 8, 32])
@pytest.mark.parametrize("kind,q", SUBS)
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_pcg_ssor_fixed_iterations(orc, h, s, kind, q, eta):
    if kind in ("hybrid", "bglobal") and s % q:
        pytest.skip("q must divide s")
    A = W.diffusion_7pt_var(12, seed=8)
    cdev, co = setup(h, orc, A)
    B = W.uniform_block(A.n, s, 30 + s)
    X0 = 0.01 * W.gaussian_block(A.n, s, 40 + s)
    for k in (1, 6):
        say("pcg ssor fixed", s, kind, eta, k)
        X, info = P.bkry_pcg_ssor_solve(h, dev_csr(P, A), to_dev(B), cdev, 1.2, to_dev(X0), kind=kind, q=q,
                                        tol=0.0, maxit=k, eta=eta)
        ro = orc.bcg_ssor(A, B, co, 1.2, X0, kind=kind, q=q, tol=0.0, maxit=k, eta=eta)
        assert info["iters"] == ro["iters"] == k and info["reorth"] == ro["reorth"]
        assert rel(to_np(X), ro["X"]) < 1e-10


@pytest.mark.parametrize("kind,q", SUBS)
@pytest.mark.parametrize("eta", [0.0, 1e4, np.inf])
def test_pcg_ssor_full_solve(orc, h, kind, q, eta):
    A = W.diffusion_7pt_var(10, seed=9)
    cdev, co = setup(h, orc, A)
    B = W.uniform_block(A.n, 4, 7)
    say("pcg ssor full", kind, eta)
    X, info = P.bkry_pcg_ssor_solve(h, dev_csr(P, A), to_dev(B), cdev, 1.0, kind=kind, q=q, tol=1e-10,
                                    maxit=2000, eta=eta, hist_cap=2000)
    ro = orc.bcg_ssor(A, B, co, 1.0, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    assert info["converged"] and ro["converged"]
    assert abs(info["iters"] - ro["iters"]) <= 1
    k = min(len(info["hist"]), len(ro["hist"]))
    assert np.allclose(info["hist"][:k], ro["hist"][:k], rtol=1e-6, atol=1e-15)
    assert max(info["true_relres"]) <= 1.5e-10
    assert rel(to_np(X), np.linalg.solve(A.to_dense(), B)) < 1e-7
    rj = orc.bcg(A, B, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta, minv=1.0 / A.to_dense().diagonal())
    assert info["iters"] < rj["iters"]


def test_pcg_ssor_edge_cases(orc, h):
    A = W.diffusion_7pt_var(6, seed=2)
    cdev, co = setup(h, orc, A)
    Ad = dev_csr(P, A)
    B = W.uniform_block(A.n, 4, 1)
    say("pcg ssor edges")
    X, info = P.bkry_pcg_ssor_solve(h, Ad, to_dev(np.zeros_like(B)), cdev, tol=1e-10)
    assert info["converged"] and info["iters"] == 0 and np.all(to_np(X) == 0)
    with pytest.raises(P.BkryError) as e:
        P.bkry_pcg_ssor_solve(h, Ad, to_dev(B), to_dev(np.zeros(A.n, np.int32)), tol=1e-10)
    assert e.value.code == P.E_INVALID
    with pytest.raises(ValueError):
        P.bkry_pcg_ssor_solve(h, Ad, to_dev(B), to_dev(np.zeros(A.n - 1, np.int32)))


def test_pcg_ssor_full_size(orc, h):
    """The 64^3 variable-coefficient workload at its full size: 3 fixed
    iterations on 8 of its right-hand sides against the oracle, then the
    full 32-column solve to 1e-10 in fewer iterations than Jacobi."""
    A, B, _ = W.build_workload("diffusion7var_64_s32")
    Ad = dev_csr(P, A)
    cdev, co = setup(h, orc, A, seed=64)
    B8 = np.ascontiguousarray(B[:, :8])
    say("pcg ssor 64^3 fixed")
    X, info = P.bkry_pcg_ssor_solve(h, Ad, to_dev(B8), cdev, 1.0, tol=0.0, maxit=3, eta=1e4)
    ro = orc.bcg_ssor(A, B8, co, 1.0, tol=0.0, maxit=3, eta=1e4)
    assert rel(to_np(X), ro["X"]) < 1e-10
    say("pcg ssor 64^3 solve")
    Bd = to_dev(B)
    X, info = P.bkry_pcg_ssor_solve(h, Ad, Bd, cdev, 1.0, tol=1e-10, maxit=5000, eta=1e4)
    assert info["converged"] and max(info["true_relres"]) <= 2e-10
    Xj, ij = P.bkry_pcg_solve(h, Ad, Bd, P.bkry_jacobi_minv(h, Ad), tol=1e-10, maxit=5000, eta=1e4)
    assert info["iters"] < ij["iters"]
    say("pcg ssor 64^3 iters", info["iters"], "s", info["seconds"], "jacobi", ij["iters"], ij["seconds"])


@pytest.mark.parametrize("eta", [1e6, 1e7])
def test_pcg_ssor_mid_solve_renormalisation(orc, h, eta):
    """Intermediate eta where the kappa_D test fires several times mid-solve:
    the solver suspends, re-normalises the residual, forms Z = M^-1 R-bar
    again and resumes; counts and residual history follow the oracle's."""
    A = W.diffusion_7pt_var(12, seed=9)
    cdev, co = setup(h, orc, A)
    B = W.uniform_block(A.n, 16, 7)
    say("pcg ssor mid-solve renormalisation", eta)
    X, info = P.bkry_pcg_ssor_solve(h, dev_csr(P, A), to_dev(B), cdev, 1.0, tol=1e-10, maxit=2000, eta=eta,
                                    hist_cap=2000)
    ro = orc.bcg_ssor(A, B, co, 1.0, tol=1e-10, maxit=2000, eta=eta, hist_cap=2000)
    assert ro["reorth"] >= 4
    assert info["converged"] and abs(info["iters"] - ro["iters"]) <= 1
    assert abs(info["reorth"] - ro["reorth"]) <= 1
    k = min(len(info["hist"]), len(ro["hist"]))
    assert np.allclose(info["hist"][:k], ro["hist"][:k], rtol=1e-6, atol=1e-15)
    assert max(info["true_relres"]) <= 1.5e-10
    assert rel(to_np(X), np.linalg.solve(A.to_dense(), B)) < 1e-7
