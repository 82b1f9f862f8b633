"""Plain FP64 CPU oracle for the block Krylov hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2104_02494_amd``)
never does, and the two share no code: the oracle is the C file
``bkry_oracle.c`` (plain loops, gcc -O2 -ffp-contract=off), written from the
thesis' definitions and algorithms, wrapped here with ctypes.

Pinning: every function below is checked by the CPU tests in ``tests/`` against
something other than itself (dense numpy/scipy linear algebra, closed forms,
invariants, brute-force minimisers on tiny inputs).  See each test module for
which pin covers which function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bkry_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PARALLEL, GLOBAL, BLOCK, HYBRID = 0, 1, 2, 3
KINDS = {"parallel": PARALLEL, "global": GLOBAL, "block": BLOCK, "hybrid": HYBRID, "bglobal": 4}
OK, NOT_CONVERGED, E_INVALID, E_BREAKDOWN, E_NONFINITE = 0, 1, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32, dbl, ptr = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        sig = {
            "or_spmm": (None, [i64, ptr, ptr, ptr, i32, ptr, ptr]),
            "or_residual": (None, [i64, ptr, ptr, ptr, i32, ptr, ptr, ptr]),
            "or_gram": (None, [i64, i32, ptr, i64, ptr, i64, ptr]),
            "or_project": (None, [i32, i32, i32, ptr]),
            "or_bdot": (i32, [i64, i32, i32, i32, ptr, ptr, ptr]),
            "or_householder_qr": (i32, [i64, i32, ptr, i64, ptr, i64, ptr]),
            "or_normalize": (i32, [i64, i32, i32, i32, ptr, ptr, ptr]),
            "or_chol_solve": (i32, [i32, i32, i32, ptr, ptr, ptr]),
            "or_sym_eigenvalues": (i32, [i32, ptr, ptr]),
            "or_kappa_D": (dbl, [i32, ptr]),
            "or_reortho_fires": (i32, [dbl, dbl, dbl]),
            "or_bcg": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, ptr, ptr, ptr, i32,
                             ptr, ptr, i32, ptr]),
            "or_color_greedy": (i32, [i64, ptr, ptr, ptr, ptr]),
            "or_ssor_apply": (i32, [i64, ptr, ptr, ptr, ptr, i32, dbl, i32, ptr, ptr]),
            "or_bcg_ssor": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, ptr, ptr, ptr,
                                  i32, ptr, i32, dbl]),
            "or_bcg1r": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, ptr, ptr, ptr, i32,
                               ptr]),
            "or_bcg_gropp": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, ptr, ptr, ptr, i32,
                               ptr]),
            "or_lu_solve": (i32, [i32, i32, i32, ptr, ptr, ptr]),
            "or_bbicgstab": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, ptr, ptr, ptr,
                                   i32]),
            "or_bbicgstab_restarted": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, dbl, dbl, i32,
                                             ptr, ptr, ptr, i32]),
            "or_block_arnoldi": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, i32, ptr, ptr, ptr]),
            "or_bgmres": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, i32, ptr, ptr, ptr, i32]),
            "or_bgmres_pipelined": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, ptr, dbl, i32, i32, i32, ptr, ptr,
                                          ptr, i32]),
            "or_block_arnoldi_pipelined": (i32, [i64, ptr, ptr, ptr, i32, i32, i32, ptr, i32, i32, ptr, ptr, ptr]),
            "or_sddmm": (None, [i64, ptr, ptr, i32, dbl, ptr, ptr, ptr]),
            "or_csr_transpose": (None, [i64, ptr, ptr, ptr, ptr, ptr, ptr, ptr]),
            "or_eps_f64": (dbl, []),
            "or_eps_f32": (dbl, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _kind(kind):
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def _csr(A):
    return A.n, _i32(A.rowptr), _i32(A.colind), _f64(A.val)


def spmm(A, X):
    n, rp, ci, v = _csr(A)
    X = _f64(X)
    s = X.shape[1]
    Y = np.empty((n, s))
    lib().or_spmm(n, _p(rp), _p(ci), _p(v), s, _p(X), _p(Y))
    return Y


def residual(A, B, X):
    n, rp, ci, v = _csr(A)
    B, X = _f64(B), _f64(X)
    R = np.empty_like(B)
    lib().or_residual(n, _p(rp), _p(ci), _p(v), B.shape[1], _p(B), _p(X), _p(R))
    return R


def gram(X, Y):
    X, Y = _f64(X), _f64(Y)
    s = X.shape[1]
    G = np.empty((s, s))
    lib().or_gram(X.shape[0], s, _p(X), s, _p(Y), s, _p(G))
    return G


def project(G, kind, q=1):
    G = _f64(G).copy()
    lib().or_project(G.shape[0], _kind(kind), q, _p(G))
    return G


def bdot(X, Y, kind, q=1):
    X, Y = _f64(X), _f64(Y)
    s = X.shape[1]
    G = np.empty((s, s))
    st = lib().or_bdot(X.shape[0], s, _kind(kind), q, _p(X), _p(Y), _p(G))
    if st != OK:
        raise ValueError("or_bdot: invalid arguments")
    return G


def householder_qr(X):
    X = _f64(X)
    m, c = X.shape
    Q = np.empty((m, c))
    R = np.empty((c, c))
    st = lib().or_householder_qr(m, c, _p(X), c, _p(Q), c, _p(R))
    if st != OK:
        raise ValueError("or_householder_qr: invalid arguments")
    return Q, R


def normalize(X, kind, q=1):
    X = _f64(X)
    n, s = X.shape
    Y = np.empty_like(X)
    N = np.empty((s, s))
    st = lib().or_normalize(n, s, _kind(kind), q, _p(X), _p(Y), _p(N))
    if st != OK:
        raise ValueError("or_normalize: invalid arguments")
    return Y, N


def chol_solve(A, B, kind, q=1):
    A, B = _f64(A), _f64(B)
    s = A.shape[0]
    X = np.empty((s, s))
    st = lib().or_chol_solve(s, _kind(kind), q, _p(A), _p(B), _p(X))
    return st, X


def sym_eigenvalues(A):
    A = _f64(A)
    ev = np.empty(A.shape[0])
    lib().or_sym_eigenvalues(A.shape[0], _p(A), _p(ev))
    return ev


def kappa_D(alpha):
    alpha = _f64(alpha)
    return lib().or_kappa_D(alpha.shape[0], _p(alpha))


def reortho_fires(eta, kappa, eps):
    return bool(lib().or_reortho_fires(float(eta), float(kappa), float(eps)))


def eps_f64():
    return lib().or_eps_f64()


def eps_f32():
    return lib().or_eps_f32()


def bcg(A, B, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, eta=0.0, eps=None, hist_cap=0,
        record_blocks=0, minv=None):
    """Adaptive block CG, preconditioned by the diagonal M with M^-1 = diag(minv)
    (minv=None: M = I).  Returns dict(status, X, iters, reorth, converged,
    relres, hist, Pk, Rk)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    Pk = np.zeros((record_blocks, n, s)) if record_blocks else None
    Rk = np.zeros((record_blocks, n, s)) if record_blocks else None
    eps = eps_f64() if eps is None else eps
    mv = None if minv is None else _f64(minv)
    if mv is not None and mv.shape != (n,):
        raise ValueError("minv must hold n entries")
    st = lib().or_bcg(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, eta, eps,
                      _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap,
                      _p(Pk), _p(Rk), record_blocks, _p(mv))
    it = int(info[0])
    return dict(status=st, X=X, iters=it, reorth=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None,
                Pk=Pk[:min(it, record_blocks)] if record_blocks else None,
                Rk=Rk[:min(it, record_blocks)] if record_blocks else None)


def color_greedy(A, prio):
    """Greedy colouring in decreasing priority (prio: n uint32).  Returns
    (colors int32[n], ncolors)."""
    n, rp, ci, _ = _csr(A)
    pr = np.ascontiguousarray(prio, dtype=np.uint32)
    if pr.shape != (n,):
        raise ValueError("prio must hold n entries")
    colors = np.zeros(n, dtype=np.int32)
    nc = lib().or_color_greedy(n, _p(rp), _p(ci), _p(pr), _p(colors))
    return colors, nc


def ssor_apply(A, colors, omega, R):
    """Z = M^-1 R for the multicolour SSOR preconditioner.  Returns (status, Z)."""
    n, rp, ci, v = _csr(A)
    R = _f64(R)
    cl = np.ascontiguousarray(colors, dtype=np.int32)
    Z = np.zeros_like(R)
    st = lib().or_ssor_apply(n, _p(rp), _p(ci), _p(v), _p(cl), int(cl.max()) + 1 if n else 0, float(omega),
                             R.shape[1], _p(R), _p(Z))
    return st, Z


def bcg_ssor(A, B, colors, omega, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, eta=0.0, eps=None,
             hist_cap=0):
    """Block CG preconditioned by multicolour SSOR.  Returns dict(status, X,
    iters, reorth, converged, relres, hist)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    cl = np.ascontiguousarray(colors, dtype=np.int32)
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    eps = eps_f64() if eps is None else eps
    st = lib().or_bcg_ssor(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, eta, eps,
                           _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap, _p(cl),
                           int(cl.max()) + 1, float(omega))
    it = int(info[0])
    return dict(status=st, X=X, iters=it, reorth=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None)


def bcg1r(A, B, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, eta=0.0, eps=None, hist_cap=0, minv=None):
    """Block CG with one reduction per iteration (alg:1R-CG), preconditioned
    by M^-1 = diag(minv) (None: M = I).  Returns dict(status, X, iters,
    reorth, converged, relres, hist)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    eps = eps_f64() if eps is None else eps
    mv = None if minv is None else _f64(minv)
    if mv is not None and mv.shape != (n,):
        raise ValueError("minv must hold n entries")
    st = lib().or_bcg1r(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, eta, eps,
                        _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap, _p(mv))
    it = int(info[0])
    return dict(status=st, X=X, iters=it, reorth=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None)


def bcg_gropp(A, B, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, eta=0.0, eps=None, hist_cap=0, minv=None):
    """Gropp's block CG (alg:gropps_block_cg: Q and Z by recurrences),
    preconditioned by M^-1 = diag(minv) (None: M = I).  Returns dict(status,
    X, iters, reorth, converged, relres, hist)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    eps = eps_f64() if eps is None else eps
    mv = None if minv is None else _f64(minv)
    if mv is not None and mv.shape != (n,):
        raise ValueError("minv must hold n entries")
    st = lib().or_bcg_gropp(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, eta, eps,
                        _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap, _p(mv))
    it = int(info[0])
    return dict(status=st, X=X, iters=it, reorth=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None)


def lu_solve(A, B, kind, q=1):
    A, B = _f64(A), _f64(B)
    X = np.zeros_like(A)
    st = lib().or_lu_solve(A.shape[0], _kind(kind), q, _p(A), _p(B), _p(X))
    return st, X


def bbicgstab(A, B, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, eta=0.0, eps=None, hist_cap=0,
              max_restarts=None):
    """Block BiCGStab with adaptive residual re-orthonormalisation (M = I);
    with max_restarts (an int >= 0) restarted on the true residual until it
    meets tol.  Returns dict(status, X, iters, reorth, converged, relres,
    hist, restarts)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    eps = eps_f64() if eps is None else eps
    if max_restarts is None:
        st = lib().or_bbicgstab(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, eta, eps,
                                _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap)
    else:
        st = lib().or_bbicgstab_restarted(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit,
                                          eta, eps, int(max_restarts), _p(info), _p(relres),
                                          _p(hist) if hist_cap else None, hist_cap)
    it = int(info[0])
    return dict(status=st, X=X, iters=it, reorth=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None, restarts=int(info[3]))


def block_arnoldi(A, R, m, kind="block", q=1, pipelined=None):
    """Block Arnoldi with modified Gram-Schmidt, or with the pipelined
    Gram-Schmidt of window `pipelined` (an int >= 0)."""
    n, rp, ci, v = _csr(A)
    R = _f64(R)
    s = R.shape[1]
    V = np.zeros((m + 1, n, s))
    H = np.zeros((m + 1, m, s, s))
    sig0 = np.zeros((s, s))
    if pipelined is None:
        st = lib().or_block_arnoldi(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(R), m, _p(V), _p(H), _p(sig0))
    else:
        st = lib().or_block_arnoldi_pipelined(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(R), m,
                                              int(pipelined), _p(V), _p(H), _p(sig0))
    return st, V, H, sig0


def bgmres(A, B, X0=None, kind="block", q=1, tol=1e-10, maxit=1000, restart=30, hist_cap=0, pipelined=None):
    """Restarted block GMRes (modified Gram-Schmidt, or the pipelined
    Gram-Schmidt of window `pipelined`).  Returns dict(status, X, iters,
    cycles, converged, relres, hist)."""
    n, rp, ci, v = _csr(A)
    B = _f64(B)
    s = B.shape[1]
    X = np.zeros_like(B) if X0 is None else _f64(X0).copy()
    info = np.zeros(4, dtype=np.int32)
    relres = np.zeros(s)
    hist = np.zeros(max(hist_cap, 1))
    if pipelined is None:
        st = lib().or_bgmres(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit, restart,
                             _p(info), _p(relres), _p(hist) if hist_cap else None, hist_cap)
    else:
        st = lib().or_bgmres_pipelined(n, _p(rp), _p(ci), _p(v), s, _kind(kind), q, _p(B), _p(X), tol, maxit,
                                       restart, int(pipelined), _p(info), _p(relres),
                                       _p(hist) if hist_cap else None, hist_cap)
    it = int(info[0])
    return dict(status=st, X=X, iters=it, cycles=int(info[1]), converged=bool(info[2]), relres=relres,
                hist=hist[:min(it, hist_cap)] if hist_cap else None)


def sddmm(A, L, X, alpha=-1.0):
    n, rp, ci, _ = _csr(A)
    L, X = _f64(L), _f64(X)
    out = np.empty(A.nnz)
    lib().or_sddmm(n, _p(rp), _p(ci), L.shape[1], alpha, _p(L), _p(X), _p(out))
    return out


def csr_transpose(A):
    n, rp, ci, v = _csr(A)
    rpT = np.empty(n + 1, dtype=np.int32)
    ciT = np.empty(A.nnz, dtype=np.int32)
    vT = np.empty(A.nnz)
    perm = np.empty(A.nnz, dtype=np.int32)
    lib().or_csr_transpose(n, _p(rp), _p(ci), _p(v), _p(rpT), _p(ciT), _p(vT), _p(perm))
    return rpT, ciT, vT, perm


def adjoint(A, X, grad_X, AT=None, kind="block", q=1, tol=1e-13, maxit=5000, eta=0.0):
    """Adjoint of the block solve A X = B for a loss with gradient grad_X:
    Lambda = A^-T grad_X (oracle block CG on A^T; A^T = A for symmetric A),
    dL/dB = Lambda, dL/dval = -(Lambda X^T) on the pattern of A."""
    AT = A if AT is None else AT
    r = bcg(AT, grad_X, kind=kind, q=q, tol=tol, maxit=maxit, eta=eta)
    lam = r["X"]
    return lam, sddmm(A, lam, X, -1.0), r
