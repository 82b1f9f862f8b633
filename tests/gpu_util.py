"""Helpers for the GPU parity tests: device handles, host<->device copies and
tolerances derived from the arithmetic (forward error bounds)."""
import sys

import numpy as np
import pytest

EPS = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a lost box)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev_csr(P, A, device="cuda"):
    return P.CsrMatrix.from_numpy(A.n, A.rowptr, A.colind, A.val, device=device)


def to_dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def to_np(t):
    return t.detach().cpu().numpy()


def spmm_bound(A, X, eps=EPS):
    """Elementwise bound gamma_k * (|A| |X|) for a k-term dot product
    (Higham, Accuracy and Stability, Sec. 3.1), k = max non-zeros per row."""
    k = int(np.diff(A.rowptr).max(initial=1))
    gamma = 1.01 * k * eps / (1 - k * eps)
    absA = type(A)(A.n, A.rowptr, A.colind, np.abs(A.val))
    import oracle
    return gamma * oracle.spmm(absA, np.abs(X)) + 1e-300


def gram_bound(X, Y, eps=EPS):
    n = X.shape[0]
    gamma = 1.01 * n * eps
    return gamma * (np.abs(X).T @ np.abs(Y)) + 1e-300


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def h():
    import paper_2104_02494_amd as P
    hd = P.Handle()
    yield hd
    hd.close()
