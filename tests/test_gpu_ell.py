"""GPU parity of the padded row-major (ELL) SpMM path against the oracle and
against the CSR path.

The ELL copy of bkry_spmm keeps each row's entries in CSR order (padding
adds nothing), so that product must reproduce the oracle bit for bit on
integer data and the CSR kernel bit for bit on any data.  The solvers' copy
moves each row's diagonal entry to the front (the fused SpMM and Gram reads
a row's own values from that entry's gather; a row without one keeps CSR
order, and the kernel then loads the own rows): their solves agree with the
CSR path to rounding."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev_csr, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")

WIDTHS = [1, 2, 3, 4, 5, 8, 16, 32]


@pytest.fixture(scope="module")
def hh():
    """Three handles: AUTO, forced CSR, forced ELL."""
    hs = {}
    for f in ("auto", "csr", "ell"):
        hs[f] = P.Handle()
        P.bkry_set_spmm_format(hs[f], f)
    yield hs
    for hd in hs.values():
        hd.close()


@pytest.mark.parametrize("s", WIDTHS)
def test_ell_spmm_integer_bit_exact(orc, hh, s):
    n = 3000
    # irregular rows (Bernoulli pattern), empty rows, ragged tail of the last tile
    A = W.random_csr(n, n, 3.0 / n, seed=40 + s, integer=True, empty_rows=(0, 17, n - 1))
    X = np.random.default_rng(s).integers(-8, 9, size=(n, s)).astype(np.float64)
    say("ell spmm int", n, s)
    Y = to_np(P.bkry_spmm(hh["ell"], dev_csr(P, A), to_dev(X)))
    assert np.array_equal(Y, orc.spmm(A, X))


@pytest.mark.parametrize("s", [8, 16])
@pytest.mark.parametrize("mat", ["laplace2d_90", "laplace3d_20"])
def test_ell_spmm_gangs_integer_bit_exact(orc, hh, s, mat):
    """Sizes whose launch width is a multiple of 64 workgroups, so that the
    rows are swept by gangs of workgroups (with a ragged last tile)."""
    A = W.laplace_2d(90) if mat == "laplace2d_90" else W.laplace_3d(20)
    X = np.random.default_rng(s).integers(-8, 9, size=(A.n, s)).astype(np.float64)
    say("ell gangs int", mat, s)
    Ad, Xd = dev_csr(P, A), to_dev(X)
    Ye = to_np(P.bkry_spmm(hh["ell"], Ad, Xd))
    assert np.array_equal(Ye, orc.spmm(A, X))
    Xg = W.gaussian_block(A.n, s, 3)
    Ye = to_np(P.bkry_spmm(hh["ell"], Ad, to_dev(Xg)))
    Yc = to_np(P.bkry_spmm(hh["csr"], Ad, to_dev(Xg)))
    assert np.array_equal(Ye.view(np.uint64), Yc.view(np.uint64))


@pytest.mark.parametrize("s", WIDTHS)
@pytest.mark.parametrize("mat", ["diffusion27", "random"])
def test_ell_spmm_matches_csr_bitwise(hh, s, mat):
    if mat == "diffusion27":
        A = W.diffusion_27pt(12, seed=7)        # 27 entries per row: several ELL chunks per row
    else:
        A = W.random_csr(3000, 3000, 9.0 / 3000, seed=11)
    X = W.gaussian_block(A.n, s, s)
    say("ell vs csr", mat, s)
    Ad, Xd = dev_csr(P, A), to_dev(X)
    Ye = to_np(P.bkry_spmm(hh["ell"], Ad, Xd))
    Yc = to_np(P.bkry_spmm(hh["csr"], Ad, Xd))
    assert np.array_equal(Ye.view(np.uint64), Yc.view(np.uint64))


@pytest.mark.parametrize("s", [4, 8, 16])
def test_ell_spmm_f32_matches_csr_bitwise(hh, s):
    A = W.laplace_3d(10)
    X = W.gaussian_block(A.n, s, 1).astype(np.float32)
    say("ell f32", s)
    Ad, Xd, v32 = dev_csr(P, A), to_dev(X), to_dev(A.val.astype(np.float32))
    Ye = to_np(P.bkry_spmm_f32(hh["ell"], Ad, v32, Xd))
    Yc = to_np(P.bkry_spmm_f32(hh["csr"], Ad, v32, Xd))
    assert np.array_equal(Ye.view(np.uint32), Yc.view(np.uint32))


def test_ell_bad_index_raises(hh):
    A = W.laplace_2d(8)
    ci = A.colind.copy()
    ci[5] = 10_000
    say("ell bad index")
    with pytest.raises(P.BkryError):
        P.bkry_spmm(hh["ell"], dev_csr(P, W.Csr(A.n, A.rowptr, ci, A.val)), to_dev(np.ones((A.n, 4))))
    with pytest.raises(P.BkryError):
        P.bkry_cg_solve(hh["auto"], dev_csr(P, W.Csr(A.n, A.rowptr, ci, A.val)), to_dev(np.ones((A.n, 4))),
                        maxit=3)


@pytest.mark.parametrize("kind,q", [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1)])
@pytest.mark.parametrize("eta", [0.0, np.inf])
def test_cg_formats_agree(hh, kind, q, eta):
    """Fixed iteration counts: CSR and ELL agree to rounding; AUTO streams
    the same ELL copy as the forced format, bit for bit.  Converged solves
    take the same number of iterations."""
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("cg formats", kind, eta)
    Ad, Bd = dev_csr(P, A), to_dev(B)
    out = {}
    for f in ("csr", "ell", "auto"):
        X, info = P.bkry_cg_solve(hh[f], Ad, Bd, kind=kind, q=q, tol=0.0, maxit=40, eta=eta)
        out[f] = to_np(X)
    say("  rel diff", rel(out["ell"], out["csr"]))
    assert rel(out["ell"], out["csr"]) <= 1e-11
    assert np.array_equal(out["ell"], out["auto"])
    its = {f: P.bkry_cg_solve(hh[f], Ad, Bd, kind=kind, q=q, tol=1e-10, maxit=2000, eta=eta)[1]["iters"]
           for f in ("csr", "ell")}
    assert its["csr"] == its["ell"]


def shuffled_dup_diag(A, seed):
    """A with every row's entries in a random order and the diagonal entry of
    every third row split into two halves (a duplicate entry)."""
    rng = np.random.default_rng(seed)
    rp, ci, va = [0], [], []
    for i in range(A.n):
        c = list(A.colind[A.rowptr[i]:A.rowptr[i + 1]])
        v = list(A.val[A.rowptr[i]:A.rowptr[i + 1]])
        if i % 3 == 0:
            d = c.index(i)
            v[d] *= 0.5
            c.append(i)
            v.append(v[d])
        o = rng.permutation(len(c))
        ci += [c[t] for t in o]
        va += [v[t] for t in o]
        rp.append(len(ci))
    return W.Csr(A.n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


@pytest.mark.parametrize("s", [8, 16])
def test_cg_formats_agree_diagonal_anywhere(hh, s):
    """Diagonal entries at every position of a row, and duplicated: the ELL
    copy puts the first in slot 0, and the fused SpMM and Gram takes the own
    rows from it."""
    A0 = W.laplace_2d(40)
    A = shuffled_dup_diag(A0, seed=s)
    B = W.uniform_block(A.n, s, s)
    say("cg formats, shuffled rows", s)
    Ad, Bd = dev_csr(P, A), to_dev(B)
    Xc, _ = P.bkry_cg_solve(hh["csr"], Ad, Bd, tol=0.0, maxit=30, eta=1e4)
    Xe, _ = P.bkry_cg_solve(hh["ell"], Ad, Bd, tol=0.0, maxit=30, eta=1e4)
    Xc, Xe = to_np(Xc), to_np(Xe)
    say("  rel diff", rel(Xe, Xc))
    assert rel(Xe, Xc) <= 1e-11
    Xs, info = P.bkry_cg_solve(hh["ell"], Ad, Bd, tol=1e-10, maxit=2000, eta=1e4)
    assert info["converged"] and rel(to_np(Xs), np.linalg.solve(A0.to_dense(), B)) < 1e-8


def test_cg_full_size_formats_agree(hh):
    """The 128^3 Laplacian with 8 right-hand sides, 3 iterations, in the
    launch configuration of the benchmark (AUTO streams the ELL copy).  The
    two SpMM kernels may run at different launch widths here (their register
    use differs, and every workgroup must be resident), which regroups the
    Gram partial sums: agreement to rounding, not bit for bit."""
    A, B, _ = W.build_workload("laplace3d_128_s8")
    say("cg 128^3 formats")
    Ad, Bd = dev_csr(P, A), to_dev(B)
    Xc, ic = P.bkry_cg_solve(hh["csr"], Ad, Bd, tol=0.0, maxit=3, eta=1e4)
    Xa, ia = P.bkry_cg_solve(hh["auto"], Ad, Bd, tol=0.0, maxit=3, eta=1e4)
    assert ic["iters"] == ia["iters"] == 3
    Xc, Xa = to_np(Xc), to_np(Xa)
    assert np.linalg.norm(Xc - Xa) <= 1e-12 * np.linalg.norm(Xc)


def test_ir_formats_agree(hh):
    A, B, _ = W.build_workload("poisson2d_32x32_s4")
    say("ir formats")
    Ad, Bd = dev_csr(P, A), to_dev(B)
    Xc, ic = P.bkry_cg_solve(hh["csr"], Ad, Bd, tol=1e-10, maxit=2000, eta=np.inf, prec=P.F32_IR)
    Xe, ie = P.bkry_cg_solve(hh["ell"], Ad, Bd, tol=1e-10, maxit=2000, eta=np.inf, prec=P.F32_IR)
    assert ic["converged"] and ie["converged"] and abs(ic["iters"] - ie["iters"]) <= 1
    say("  rel diff", rel(to_np(Xe), to_np(Xc)))
    assert rel(to_np(Xe), to_np(Xc)) <= 1e-9


def test_gmres_formats_agree(hh):
    A = W.convdiff_2d(24)
    B = W.gaussian_block(A.n, 4, 5)
    say("gmres formats")
    Ad, Bd = dev_csr(P, A), to_dev(B)
    Xc, ic = P.bkry_gmres_solve(hh["csr"], Ad, Bd, tol=0.0, maxit=20, restart=10)
    Xe, ie = P.bkry_gmres_solve(hh["ell"], Ad, Bd, tol=0.0, maxit=20, restart=10)
    assert ic["iters"] == ie["iters"]
    say("  rel diff", rel(to_np(Xe), to_np(Xc)))
    assert rel(to_np(Xe), to_np(Xc)) <= 1e-11
    Xc, ic = P.bkry_gmres_solve(hh["csr"], Ad, Bd, tol=1e-10, maxit=60, restart=10)
    Xe, ie = P.bkry_gmres_solve(hh["ell"], Ad, Bd, tol=1e-10, maxit=60, restart=10)
    assert ic["iters"] == ie["iters"]


def test_gmres_formats_agree_without_diagonal(hh):
    """A row without a diagonal entry (kept in CSR order in the solvers' ELL
    copy, the other rows diagonal first): the iterates agree with the CSR
    path's to rounding."""
    A0 = W.convdiff_2d(24)
    keep = np.ones(A0.nnz, bool)
    r = 100
    keep[A0.rowptr[r] + list(A0.colind[A0.rowptr[r]:A0.rowptr[r + 1]]).index(r)] = False
    cnt = np.diff(A0.rowptr) - np.bincount(np.repeat(np.arange(A0.n), np.diff(A0.rowptr))[~keep], minlength=A0.n)
    A = W.Csr(A0.n, np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32), A0.colind[keep], A0.val[keep])
    B = W.gaussian_block(A.n, 4, 5)
    say("gmres formats, row without diagonal")
    Ad, Bd = dev_csr(P, A), to_dev(B)
    Xc, ic = P.bkry_gmres_solve(hh["csr"], Ad, Bd, tol=0.0, maxit=20, restart=10)
    Xe, ie = P.bkry_gmres_solve(hh["ell"], Ad, Bd, tol=0.0, maxit=20, restart=10)
    assert ic["iters"] == ie["iters"]
    say("  rel diff", rel(to_np(Xe), to_np(Xc)))
    assert rel(to_np(Xe), to_np(Xc)) <= 1e-11
