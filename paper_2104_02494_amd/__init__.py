"""Python binding of libbkry.so, the MI355X block Krylov library.

Argument marshalling only: every function passes torch device tensors as raw
pointers to the C ABI declared in ``include/bkry.h`` (same names) and
returns what the library wrote.  All arithmetic runs in the HIP kernels of
the library; there is no CPU fallback -- if the library is missing, every
call raises.

Block vectors are torch tensors of shape (n, p), row-major, float64 (float32
for the ``_f32`` kernels), on the handle's device.  CSR matrices are
``CsrMatrix`` objects holding int32 row pointers / column indices and float64
values on the device.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BKRY_LIB") or os.path.join(_HERE, "libbkry.so")

OK, NOT_CONVERGED, E_INVALID, E_BREAKDOWN, E_NONFINITE, E_HIP, E_ALLOC = 0, 1, -1, -2, -3, -4, -5
PARALLEL, GLOBAL, BLOCK, HYBRID, BLOCK_GLOBAL = 0, 1, 2, 3, 4
KINDS = {"parallel": PARALLEL, "global": GLOBAL, "block": BLOCK, "hybrid": HYBRID, "bglobal": BLOCK_GLOBAL}
F64, F32_IR = 0, 1
_CODES = {E_INVALID: "invalid argument", E_BREAKDOWN: "breakdown", E_NONFINITE: "non-finite",
          E_HIP: "HIP error", E_ALLOC: "allocation failure"}


class BkryError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class bkry_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class bkry_subalg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q", ctypes.c_int32)]


class bkry_info(ctypes.Structure):
    _fields_ = [("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("hist_cap", ctypes.c_int32),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("relres", ctypes.POINTER(ctypes.c_double)),
                ("true_relres", ctypes.POINTER(ctypes.c_double)),
                ("iters", ctypes.c_int32), ("reorth", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("hist_len", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


EXPORTS = ["bkry_create", "bkry_destroy", "bkry_set_stream", "bkry_synchronize", "bkry_last_error",
           "bkry_profile", "bkry_profile_read", "bkry_set_spmm_format", "bkry_spmm",
           "bkry_spmm_f32", "bkry_bdot", "bkry_bdot_f32", "bkry_tsqr", "bkry_cg_solve", "bkry_pcg_solve",
           "bkry_cg1r_solve", "bkry_color", "bkry_ssor_apply", "bkry_pcg_ssor_solve", "bkry_jacobi_minv", "bkry_bicgstab_solve", "bkry_gmres_solve", "bkry_sddmm", "bkry_csr_transpose", "bkry_bdot_noalloc", "bkry_gmres_pipelined_solve", "bkry_gropp_solve"]

_lib = None


def lib():
    """Load libbkry.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        H = ctypes.c_void_p
        csr_p = ctypes.POINTER(bkry_csr)
        info_p = ctypes.POINTER(bkry_info)
        sig = {
            "bkry_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, vp],
            "bkry_destroy": [H],
            "bkry_set_stream": [H, vp],
            "bkry_synchronize": [H],
            "bkry_profile": [H, ctypes.c_int],
            "bkry_profile_read": [H, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32],
            "bkry_set_spmm_format": [H, i32],
            "bkry_spmm": [H, csr_p, i32, vp, vp],
            "bkry_spmm_f32": [H, i64, i64, vp, vp, vp, i32, vp, vp],
            "bkry_bdot": [H, i64, i32, bkry_subalg, vp, vp, vp],
            "bkry_bdot_f32": [H, i64, i32, bkry_subalg, vp, vp, vp],
            "bkry_bdot_noalloc": [H, i64, i32, bkry_subalg, vp, vp, vp],
            "bkry_tsqr": [H, i64, i32, bkry_subalg, vp, vp],
            "bkry_cg_solve": [H, csr_p, i32, bkry_subalg, vp, vp, dbl, i32, dbl, i32, info_p],
            "bkry_pcg_solve": [H, csr_p, i32, bkry_subalg, vp, vp, vp, dbl, i32, dbl, info_p],
            "bkry_cg1r_solve": [H, csr_p, i32, bkry_subalg, vp, vp, dbl, i32, dbl, info_p],
            "bkry_gropp_solve": [H, csr_p, i32, bkry_subalg, vp, vp, vp, dbl, i32, dbl, info_p],
            "bkry_color": [H, csr_p, vp, vp, ctypes.POINTER(i32)],
            "bkry_ssor_apply": [H, csr_p, i32, vp, dbl, vp, vp],
            "bkry_pcg_ssor_solve": [H, csr_p, i32, bkry_subalg, vp, vp, vp, dbl, dbl, i32, dbl, info_p],
            "bkry_jacobi_minv": [H, csr_p, vp],
            "bkry_bicgstab_solve": [H, csr_p, i32, bkry_subalg, vp, vp, dbl, i32, dbl, info_p],
            "bkry_gmres_solve": [H, csr_p, i32, bkry_subalg, vp, vp, dbl, i32, i32, info_p],
            "bkry_gmres_pipelined_solve": [H, csr_p, i32, bkry_subalg, vp, vp, dbl, i32, i32, i32, info_p],
            "bkry_sddmm": [H, csr_p, i32, dbl, vp, vp, vp],
            "bkry_csr_transpose": [H, csr_p, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.bkry_last_error.argtypes = [H]
        L.bkry_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _subalg(kind, q=1):
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    return bkry_subalg(k, int(q))


class Handle:
    """Owns a bkry handle on one device; work is ordered on torch's current stream."""

    def __init__(self, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the block Krylov library needs an MI355X")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream(self.device).cuda_stream
            rc = lib().bkry_create(ctypes.byref(h), self.device.index, ctypes.c_void_p(st))
        if rc != OK:
            raise BkryError(rc, "bkry_create failed")
        self.h = h

    def _sync_stream(self):
        st = torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().bkry_set_stream(self.h, ctypes.c_void_p(st)))

    def _check(self, rc, allow=(OK,)):
        if rc in allow:
            return rc
        msg = lib().bkry_last_error(self.h).decode()
        raise BkryError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().bkry_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class CsrMatrix:
    """CSR matrix on the device: int32 rowptr[n+1], int32 colind[nnz], float64 val[nnz]."""
    n: int
    rowptr: torch.Tensor
    colind: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.colind.numel())

    @classmethod
    def from_numpy(cls, n, rowptr, colind, val, device="cuda"):
        t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
        return cls(int(n), t(rowptr, torch.int32), t(colind, torch.int32), t(val, torch.float64))

    def desc(self) -> bkry_csr:
        return bkry_csr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr() if self.nnz else None,
                        self.val.data_ptr() if self.nnz else None)


def _block(t: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
    if t.dim() != 2 or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"expected a contiguous 2-D {dtype} CUDA tensor, got {t.dtype} {tuple(t.shape)}")
    return t


def bkry_spmm(h: Handle, A: CsrMatrix, X: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
    """Y = A X (asynchronous on the current stream)."""
    _block(X)
    Y = torch.empty_like(X) if Y is None else _block(Y)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_spmm(h.h, ctypes.byref(d), X.shape[1], _ptr(X), _ptr(Y)))
    return Y


def bkry_spmm_f32(h: Handle, A: CsrMatrix, val32: torch.Tensor, X: torch.Tensor, Y=None) -> torch.Tensor:
    _block(X, torch.float32)
    Y = torch.empty_like(X) if Y is None else _block(Y, torch.float32)
    h._sync_stream()
    h._check(lib().bkry_spmm_f32(h.h, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(val32), X.shape[1],
                                 _ptr(X), _ptr(Y)))
    return Y


def bkry_bdot(h: Handle, X: torch.Tensor, Y: torch.Tensor, kind="block", q=1) -> torch.Tensor:
    """G = <X, Y>_S (p x p, float64, on the device)."""
    f32 = X.dtype == torch.float32
    _block(X, X.dtype)
    _block(Y, X.dtype)
    p = X.shape[1]
    G = torch.empty((p, p), dtype=torch.float64, device=X.device)
    h._sync_stream()
    fn = lib().bkry_bdot_f32 if f32 else lib().bkry_bdot
    h._check(fn(h.h, X.shape[0], p, _subalg(kind, q), _ptr(X), _ptr(Y), _ptr(G)))
    return G


def bkry_bdot_noalloc(h: Handle, X: torch.Tensor, Y: torch.Tensor, G: torch.Tensor, kind="block", q=1) -> torch.Tensor:
    """G = <X, Y>_S into the caller's p x p float64 device tensor G, with the
    library's fixed per-GPU scratch array instead of its workspace (the call
    allocates no device memory)."""
    _block(X)
    _block(Y)
    p = X.shape[1]
    if not (G.is_cuda and G.dtype == torch.float64 and G.is_contiguous() and tuple(G.shape) == (p, p)):
        raise ValueError("G must be a contiguous p x p float64 device tensor")
    h._sync_stream()
    h._check(lib().bkry_bdot_noalloc(h.h, X.shape[0], p, _subalg(kind, q), _ptr(X), _ptr(Y), _ptr(G)))
    return G


def bkry_tsqr(h: Handle, X: torch.Tensor, kind="block", q=1) -> torch.Tensor:
    """In place: X <- Q, returns R (p x p) with X_in = Q R, <Q,Q>_S = I."""
    _block(X)
    p = X.shape[1]
    R = torch.empty((p, p), dtype=torch.float64, device=X.device)
    h._sync_stream()
    h._check(lib().bkry_tsqr(h.h, X.shape[0], p, _subalg(kind, q), _ptr(X), _ptr(R)))
    return R


def _info(p, hist_cap, inner_tol=0.0, max_outer=0):
    hist = (ctypes.c_double * max(hist_cap, 1))()
    rel = (ctypes.c_double * p)()
    trel = (ctypes.c_double * p)()
    info = bkry_info(inner_tol, max_outer, hist_cap, hist if hist_cap else None, rel, trel)
    return info, hist, rel, trel


def _info_dict(rc, info, hist, rel, trel, p):
    return dict(status=rc, iters=info.iters, reorth=info.reorth, outer_iters=info.outer_iters,
                converged=bool(info.converged), seconds=info.seconds,
                hist=[hist[i] for i in range(info.hist_len)], relres=[rel[i] for i in range(p)],
                true_relres=[trel[i] for i in range(p)])


def bkry_cg_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, X: torch.Tensor | None = None, kind="block", q=1,
                  tol=1e-10, maxit=1000, eta=1e4, prec=F64, hist_cap=0, inner_tol=0.0, max_outer=0, minv=None):
    """Block CG with adaptive residual re-orthonormalisation; X (in/out, zeros if None).
    minv (FP64 device vector of n entries): diagonal of M^-1 of a diagonal
    preconditioner M (bkry_pcg_solve); None: no preconditioner.
    Returns (X, info).  Raises on invalid input, breakdown or non-finite values."""
    _block(B)
    X = torch.zeros_like(B) if X is None else _block(X)
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap, inner_tol, max_outer)
    h._sync_stream()
    d = A.desc()
    if minv is not None:
        if not (minv.is_cuda and minv.dtype == torch.float64 and minv.is_contiguous() and minv.numel() == A.n):
            raise ValueError("minv must be a contiguous FP64 device vector of n entries")
        if prec != F64:
            raise ValueError("the preconditioned solve runs in FP64")
        rc = lib().bkry_pcg_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), _ptr(minv),
                                  float(tol), int(maxit), float(eta), ctypes.byref(info))
    else:
        rc = lib().bkry_cg_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), float(tol),
                                 int(maxit), float(eta), int(prec), ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_pcg_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, minv: torch.Tensor, X: torch.Tensor | None = None,
                   kind="block", q=1, tol=1e-10, maxit=1000, eta=1e4, hist_cap=0):
    """Block CG with the diagonal preconditioner M^-1 = diag(minv) (FP64).  Returns (X, info)."""
    return bkry_cg_solve(h, A, B, X, kind=kind, q=q, tol=tol, maxit=maxit, eta=eta, hist_cap=hist_cap, minv=minv)


def bkry_gropp_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, X: torch.Tensor | None = None, minv=None,
                     kind="block", q=1, tol=1e-10, maxit=1000, eta=1e4, hist_cap=0):
    """Gropp's block CG (Q and Z by recurrences), FP64, with the diagonal
    preconditioner M^-1 = diag(minv) or M = I (minv None).  Returns (X, info)."""
    _block(B)
    X = torch.zeros_like(B) if X is None else _block(X)
    if minv is not None and not (minv.is_cuda and minv.dtype == torch.float64 and minv.is_contiguous()
                                 and minv.numel() == A.n):
        raise ValueError("minv must be a contiguous FP64 device vector of n entries")
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap)
    h._sync_stream()
    d = A.desc()
    rc = lib().bkry_gropp_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), _ptr(minv), float(tol),
                                int(maxit), float(eta), ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_cg1r_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, X: torch.Tensor | None = None, kind="block", q=1,
                    tol=1e-10, maxit=1000, eta=1e4, hist_cap=0):
    """Block CG with one reduction per iteration (FP64, no preconditioner);
    X (in/out, zeros if None).  Returns (X, info)."""
    _block(B)
    X = torch.zeros_like(B) if X is None else _block(X)
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap)
    h._sync_stream()
    d = A.desc()
    rc = lib().bkry_cg1r_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), float(tol), int(maxit),
                               float(eta), ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_color(h: Handle, A: CsrMatrix, prio: torch.Tensor):
    """Greedy multicolour ordering in decreasing priority (prio: uint32 device
    vector of n entries, passed as int32 storage).  Returns (colors int32
    device tensor, ncolors)."""
    if not (prio.is_cuda and prio.dtype in (torch.int32, torch.uint32) and prio.is_contiguous()
            and prio.numel() == A.n):
        raise ValueError("prio must be a contiguous 32-bit device vector of n entries")
    colors = torch.empty(A.n, dtype=torch.int32, device=A.rowptr.device)
    nc = ctypes.c_int32(0)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_color(h.h, ctypes.byref(d), _ptr(prio), _ptr(colors), ctypes.byref(nc)))
    return colors, int(nc.value)


def _colors(A, colors):
    if not (colors.is_cuda and colors.dtype == torch.int32 and colors.is_contiguous() and colors.numel() == A.n):
        raise ValueError("colors must be a contiguous int32 device vector of n entries")


def bkry_ssor_apply(h: Handle, A: CsrMatrix, colors: torch.Tensor, omega: float, R: torch.Tensor) -> torch.Tensor:
    """Z = M^-1 R for the multicolour SSOR preconditioner."""
    _block(R)
    _colors(A, colors)
    Z = torch.empty_like(R)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_ssor_apply(h.h, ctypes.byref(d), R.shape[1], _ptr(colors), float(omega), _ptr(R), _ptr(Z)))
    return Z


def bkry_pcg_ssor_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, colors: torch.Tensor, omega=1.0,
                        X: torch.Tensor | None = None, kind="block", q=1, tol=1e-10, maxit=1000, eta=1e4,
                        hist_cap=0):
    """Block CG preconditioned by multicolour SSOR (FP64).  Returns (X, info)."""
    _block(B)
    _colors(A, colors)
    X = torch.zeros_like(B) if X is None else _block(X)
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap)
    h._sync_stream()
    d = A.desc()
    rc = lib().bkry_pcg_ssor_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), _ptr(colors),
                                   float(omega), float(tol), int(maxit), float(eta), ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_jacobi_minv(h: Handle, A: CsrMatrix) -> torch.Tensor:
    """minv[i] = 1 / A_ii (the Jacobi preconditioner for bkry_cg_solve(minv=...))."""
    out = torch.empty(A.n, dtype=torch.float64, device=A.rowptr.device)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_jacobi_minv(h.h, ctypes.byref(d), _ptr(out)))
    return out


def bkry_bicgstab_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, X: torch.Tensor | None = None, kind="block",
                        q=1, tol=1e-10, maxit=1000, eta=1e4, hist_cap=0):
    """Block BiCGStab with adaptive residual re-orthonormalisation (FP64, no
    preconditioner); X (in/out, zeros if None).  Returns (X, info)."""
    _block(B)
    X = torch.zeros_like(B) if X is None else _block(X)
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap)
    h._sync_stream()
    d = A.desc()
    rc = lib().bkry_bicgstab_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), float(tol),
                                   int(maxit), float(eta), ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_gmres_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, X: torch.Tensor | None = None, kind="block", q=1,
                     tol=1e-10, maxit=1000, restart=30, hist_cap=0, pipelined=None):
    """Restarted block GMRes (TSQR Arnoldi with classical Gram-Schmidt applied
    twice, or with the pipelined Gram-Schmidt of window `pipelined` >= 1
    through bkry_gmres_pipelined_solve).  Returns (X, info)."""
    _block(B)
    X = torch.zeros_like(B) if X is None else _block(X)
    p = B.shape[1]
    info, hist, rel, trel = _info(p, hist_cap)
    h._sync_stream()
    d = A.desc()
    if pipelined is None:
        rc = lib().bkry_gmres_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X), float(tol),
                                    int(maxit), int(restart), ctypes.byref(info))
    else:
        rc = lib().bkry_gmres_pipelined_solve(h.h, ctypes.byref(d), p, _subalg(kind, q), _ptr(B), _ptr(X),
                                              float(tol), int(maxit), int(restart), int(pipelined),
                                              ctypes.byref(info))
    h._check(rc, allow=(OK, NOT_CONVERGED))
    return X, _info_dict(rc, info, hist, rel, trel, p)


def bkry_gmres_pipelined_solve(h: Handle, A: CsrMatrix, B: torch.Tensor, r: int, X: torch.Tensor | None = None,
                               kind="block", q=1, tol=1e-10, maxit=1000, restart=30, hist_cap=0):
    """Restarted block GMRes with the pipelined Gram-Schmidt of window r >= 1."""
    return bkry_gmres_solve(h, A, B, X, kind=kind, q=q, tol=tol, maxit=maxit, restart=restart, hist_cap=hist_cap,
                            pipelined=r)


def bkry_sddmm(h: Handle, A: CsrMatrix, L: torch.Tensor, X: torch.Tensor, alpha=-1.0) -> torch.Tensor:
    """out[k] = alpha * <L[i], X[j]> for the k-th stored entry (i, j) of A."""
    _block(L)
    _block(X)
    out = torch.empty(A.nnz, dtype=torch.float64, device=L.device)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_sddmm(h.h, ctypes.byref(d), L.shape[1], float(alpha), _ptr(L), _ptr(X), _ptr(out)))
    return out


def bkry_csr_transpose(h: Handle, A: CsrMatrix):
    """Returns (A^T as CsrMatrix, permT) with valT = val[permT]."""
    dev = A.rowptr.device
    rpT = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    ciT = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    vT = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    h._sync_stream()
    d = A.desc()
    h._check(lib().bkry_csr_transpose(h.h, ctypes.byref(d), _ptr(rpT), _ptr(ciT), _ptr(vT), _ptr(perm)))
    nz = A.nnz
    return CsrMatrix(A.n, rpT, ciT[:nz], vT[:nz]), perm[:nz]


def bkry_synchronize(h: Handle):
    h._check(lib().bkry_synchronize(h.h))


PROF_CG_SPMM, PROF_CG_UPDATE, PROF_CG_PUPDATE, PROF_CG_NORMALISE = 0, 1, 2, 3


FMT_AUTO, FMT_CSR, FMT_ELL = 0, 1, 2
_FMTS = {"auto": FMT_AUTO, "csr": FMT_CSR, "ell": FMT_ELL}


def bkry_set_spmm_format(h: Handle, fmt):
    """Matrix format streamed by the SpMM: "auto", "csr" or "ell" (or 0/1/2)."""
    f = _FMTS[fmt] if isinstance(fmt, str) else int(fmt)
    h._check(lib().bkry_set_spmm_format(h.h, f))


def bkry_profile(h: Handle, enable=True, kernels=None, every=1):
    """Event timing of the CG driver's streaming kernels: enable=False turns
    it off; `kernels` lists the kernel ids to time (default: all four);
    `every` times one launch in that many of each kernel."""
    if not enable:
        mask = 0
    elif kernels is None:
        mask = 0xF
    else:
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
    if mask and not 1 <= int(every) <= 255:
        raise ValueError("every must be in [1, 255]")
    h._check(lib().bkry_profile(h.h, mask | ((int(every) if mask else 0) << 8)))


def bkry_profile_read(h: Handle, kernel: int, reset: bool = False):
    """(total milliseconds, number of timed launches) of one kernel id."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    h._check(lib().bkry_profile_read(h.h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt), int(reset)))
    return ms.value, cnt.value


from .autograd import BlockSolve, block_solve  # noqa: E402,F401
