"""GPU parity of the building blocks through the C ABI: SpMM (BOP), BDOT,
TSQR normaliser, SDDMM and CSR transpose against the oracle.

Integer-valued inputs must match bit for bit; random inputs within the
forward error bounds of the summations (Higham's gamma_k)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import EPS, EPS32, dev_csr, gram_bound, h, rel, say, spmm_bound, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")

SUBS = [("block", 1), ("hybrid", 2), ("parallel", 1), ("global", 1), ("bglobal", 2)]
WIDTHS = [1, 2, 3, 4, 5, 8, 16, 32]


@pytest.mark.parametrize("s", WIDTHS)
def test_spmm_integer_bit_exact(orc, h, s):
    n = 3000
    A = W.random_csr(n, n, 3.0 / n, seed=s, integer=True, empty_rows=(0, 17, n - 1))
    X = np.random.default_rng(s).integers(-8, 9, size=(n, s)).astype(np.float64)
    say("spmm int", n, s)
    Y = to_np(P.bkry_spmm(h, dev_csr(P, A), to_dev(X)))
    assert np.array_equal(Y, orc.spmm(A, X))


@pytest.mark.parametrize("s", WIDTHS)
def test_spmm_random_within_bound(orc, h, s):
    A = W.diffusion_27pt(12, seed=7)            # 27 nnz per row, 1728 rows (several tiles + ragged tail)
    X = W.gaussian_block(A.n, s, s)
    say("spmm rnd", A.n, s)
    Y = to_np(P.bkry_spmm(h, dev_csr(P, A), to_dev(X)))
    assert np.all(np.abs(Y - orc.spmm(A, X)) <= 2 * spmm_bound(A, X))


def test_spmm_f32(orc, h):
    A = W.laplace_3d(10)
    X = W.gaussian_block(A.n, 16, 1).astype(np.float32)
    say("spmm f32")
    Y = to_np(P.bkry_spmm_f32(h, dev_csr(P, A), to_dev(A.val.astype(np.float32)), to_dev(X)))
    ref = orc.spmm(W.Csr(A.n, A.rowptr, A.colind, A.val.astype(np.float32).astype(np.float64)), X.astype(np.float64))
    assert np.all(np.abs(Y - ref) <= 2 * spmm_bound(A, X.astype(np.float64), eps=EPS32))


def test_spmm_bad_index_reported(h):
    A = W.laplace_2d(8)
    ci = A.colind.copy()
    ci[5] = 10_000
    Ab = W.Csr(A.n, A.rowptr, ci, A.val)
    say("spmm bad index")
    P.bkry_spmm(h, dev_csr(P, Ab), to_dev(np.ones((A.n, 4))))
    with pytest.raises(P.BkryError):
        P.bkry_synchronize(h)
    P.bkry_synchronize(h)                         # flag was cleared


@pytest.mark.parametrize("s", WIDTHS)
@pytest.mark.parametrize("kind,q", SUBS)
def test_bdot(orc, h, s, kind, q):
    if kind in ("hybrid", "bglobal") and s % q:
        pytest.skip("q must divide s")
    n = 70_001
    X = W.gaussian_block(n, s, 1)
    Y = W.gaussian_block(n, s, 2)
    say("bdot", n, s, kind)
    G = to_np(P.bkry_bdot(h, to_dev(X), to_dev(Y), kind, q))
    ref = orc.bdot(X, Y, kind, q)
    bound = orc.project(gram_bound(X, Y), kind if kind != "global" else "parallel", q)
    if kind == "global":
        bound = np.eye(s) * np.trace(gram_bound(X, Y)) / s
    assert np.all(np.abs(G - ref) <= bound + 1e-300)
    mask = ref == 0
    assert np.all(G[mask] == 0)


def test_bdot_integer_bit_exact(orc, h):
    rng = np.random.default_rng(3)
    X = rng.integers(-4, 5, size=(50_000, 8)).astype(np.float64)
    Y = rng.integers(-4, 5, size=(50_000, 8)).astype(np.float64)
    say("bdot int")
    assert np.array_equal(to_np(P.bkry_bdot(h, to_dev(X), to_dev(Y), "block")), X.T @ Y)


def test_bdot_f32(orc, h):
    X = W.gaussian_block(40_000, 16, 1).astype(np.float32)
    say("bdot f32")
    G = to_np(P.bkry_bdot(h, to_dev(X), to_dev(X), "block"))
    ref = X.astype(np.float64).T @ X.astype(np.float64)
    assert np.all(np.abs(G - ref) <= 2 * gram_bound(X.astype(np.float64), X.astype(np.float64), eps=EPS32))


def canon(Q, R):
    d = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * d, R * d[:, None]


@pytest.mark.parametrize("n,s", [(8, 8), (255, 4), (1000, 3), (70_000, 8), (66_000, 16), (33_000, 32), (257, 2)])
def test_tsqr_block_matches_householder(orc, h, n, s):
    X = W.gaussian_block(n, s, n + s)
    say("tsqr", n, s)
    Xd = to_dev(X)
    R = to_np(P.bkry_tsqr(h, Xd, "block"))
    Q = to_np(Xd)
    Qo, Ro = orc.householder_qr(X)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert rel(R, Ro) < 1e-12 and rel(Q, Qo) < 1e-12
    assert np.abs(Q.T @ Q - np.eye(s)).max() < 1e-13
    assert rel(Q @ R, X) < 1e-14


def test_tsqr_full_size_vs_householder(orc, h):
    """The standalone TSQR workload itself: 4,194,304 x 32 Gaussian (seed
    1044) against one Householder QR of the whole matrix in the oracle
    (about 17 GFLOP on one core), after sign canonicalisation."""
    X = W.tsqr_input()
    say("tsqr 4194304 x 32 vs householder")
    Xd = to_dev(X)
    R = to_np(P.bkry_tsqr(h, Xd, "block"))
    Q = to_np(Xd)
    del Xd
    Qo, Ro = orc.householder_qr(X)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    assert rel(R, Ro) < 1e-12 and rel(Q, Qo) < 1e-12
    assert np.abs(Q.T @ Q - np.eye(32)).max() < 1e-13
    assert rel(Q @ R, X) < 1e-13


@pytest.mark.parametrize("s", [9, 12, 16, 20, 24, 31, 32])
def test_matrix_core_widths(orc, h, s):
    """Widths 9..32 run the FP64 Gram and row products on the matrix cores
    (16 x 16 x 4 tiles, columns past s masked, ragged last tile): BDOT within
    the summation bound, the normaliser against Householder QR."""
    n = 70_001
    X = W.gaussian_block(n, s, 50 + s)
    Y = W.gaussian_block(n, s, 60 + s)
    say("matrix cores: bdot", n, s)
    G = to_np(P.bkry_bdot(h, to_dev(X), to_dev(Y), "block"))
    assert np.all(np.abs(G - orc.bdot(X, Y, "block")) <= gram_bound(X, Y) + 1e-300)
    say("matrix cores: tsqr", n, s)
    Xd = to_dev(X)
    R = to_np(P.bkry_tsqr(h, Xd, "block"))
    Q = to_np(Xd)
    Qo, Ro = orc.householder_qr(X)
    assert rel(R, Ro) < 1e-12 and rel(Q, Qo) < 1e-12
    assert np.abs(Q.T @ Q - np.eye(s)).max() < 1e-13
    for kind, q in (("hybrid", 2), ("hybrid", 4), ("bglobal", 2), ("bglobal", 4)) if s % 4 == 0 else ():
        say("matrix cores: tsqr", kind, q, s)
        Xd = to_dev(X)
        N = to_np(P.bkry_tsqr(h, Xd, kind, q))
        Yo, No = orc.normalize(X, kind, q)
        assert rel(N, No) < 1e-12 and rel(to_np(Xd), Yo) < 1e-12


@pytest.mark.parametrize("kind,q", SUBS + [("hybrid", 4), ("bglobal", 4), ("bglobal", 8)])
def test_tsqr_subalgebras(orc, h, kind, q):
    n, s = 50_000, 8
    X = W.gaussian_block(n, s, 4)
    say("tsqr sub", kind, q)
    Xd = to_dev(X)
    N = to_np(P.bkry_tsqr(h, Xd, kind, q))
    Y = to_np(Xd)
    Yo, No = orc.normalize(X, kind, q)
    assert rel(N, No) < 1e-12 and rel(Y, Yo) < 1e-12
    assert np.abs(orc.bdot(Y, Y, kind, q) - np.eye(s)).max() < 1e-13


@pytest.mark.parametrize("case", ["zero_col", "dup_col", "zero_all", "tiny_n"])
def test_tsqr_rank_deficient(orc, h, case):
    n, s = 3000, 8
    X = W.gaussian_block(n, s, 9)
    if case == "zero_col":
        X[:, 3] = 0.0
    elif case == "dup_col":
        X[:, 5] = X[:, 1]
    elif case == "zero_all":
        X[:] = 0.0
    else:
        X = X[:8].copy()
        X[:, 7] = X[:, 0] + X[:, 1]
        n = 8
    say("tsqr rank-deficient", case)
    Xd = to_dev(X)
    R = to_np(P.bkry_tsqr(h, Xd, "block"))
    Q = to_np(Xd)
    # several completions are correct: check the invariants only
    assert np.abs(Q.T @ Q - np.eye(s)).max() < 1e-12
    assert np.abs(Q @ R - X).max() <= 1e-13 * max(1.0, np.abs(X).max())
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    # the unique part: R^T R = X^T X
    assert np.abs(R.T @ R - X.T @ X).max() <= 1e-12 * max(1.0, np.abs(X.T @ X).max())


@pytest.mark.parametrize("s", [1, 4, 32])
def test_sddmm(orc, h, s):
    A = W.diffusion_7pt_var(10, seed=3)
    L = W.gaussian_block(A.n, s, 1)
    X = W.gaussian_block(A.n, s, 2)
    say("sddmm", s)
    out = to_np(P.bkry_sddmm(h, dev_csr(P, A), to_dev(L), to_dev(X), alpha=-1.0))
    ref = orc.sddmm(A, L, X, -1.0)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    bound = 1.01 * s * EPS * np.sum(np.abs(L[rows]) * np.abs(X[A.colind]), axis=1)
    assert np.all(np.abs(out - ref) <= bound + 1e-300)


def test_sddmm_integer_bit_exact(orc, h):
    A = W.random_csr(500, 500, 0.02, seed=2, integer=True, empty_rows=(3,))
    rng = np.random.default_rng(1)
    L = rng.integers(-3, 4, size=(500, 8)).astype(float)
    X = rng.integers(-3, 4, size=(500, 8)).astype(float)
    say("sddmm int")
    assert np.array_equal(to_np(P.bkry_sddmm(h, dev_csr(P, A), to_dev(L), to_dev(X))), orc.sddmm(A, L, X, -1.0))


@pytest.mark.parametrize("which", ["convdiff", "random"])
def test_csr_transpose_bit_exact(orc, h, which):
    A = W.convdiff_2d(40) if which == "convdiff" else W.random_csr(2000, 2000, 0.003, seed=5, integer=False,
                                                                    empty_rows=(0, 7))
    say("transpose", which)
    AT, perm = P.bkry_csr_transpose(h, dev_csr(P, A))
    rpT, ciT, vT, pT = orc.csr_transpose(A)
    assert np.array_equal(to_np(AT.rowptr), rpT) and np.array_equal(to_np(AT.colind), ciT)
    assert np.array_equal(to_np(AT.val), vT) and np.array_equal(to_np(perm), pT)
