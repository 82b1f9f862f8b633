"""The allocation-free BDOT (bkry_bdot_noalloc) through the C ABI against
bkry_bdot: the same kernels on a fixed per-GPU scratch array instead of the
handle's workspace, so the Grams must agree bit for bit.  Two calls in a row,
the second with a smaller input, so stale scratch contents from the first
call would show; every subalgebra; device memory use checked unchanged."""
import gc

import numpy as np
import pytest

import workloads as W
from gpu_util import h, say, to_dev, to_np  # noqa: F401

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2104_02494_amd")
torch = pytest.importorskip("torch")

CASES = [(8, "block", 1), (8, "hybrid", 2), (8, "parallel", 1), (8, "global", 1), (8, "bglobal", 2),
         (32, "block", 1), (16, "hybrid", 4), (3, "block", 1)]


@pytest.mark.parametrize("p,kind,q", CASES)
def test_noalloc_bdot_matches_bdot(h, p, kind, q):
    for n in (1_000_003, 777):                       # second call smaller
        X = to_dev(W.gaussian_block(n, p, n % 97 + p))
        Y = to_dev(W.gaussian_block(n, p, n % 89 + 2 * p))
        say("bdot_noalloc", n, p, kind, q)
        ref = to_np(P.bkry_bdot(h, X, Y, kind, q))
        G = torch.full((p, p), float("nan"), dtype=torch.float64, device=X.device)
        # no garbage collection inside the measured window: a collection could
        # free tensors of earlier tests there and move the count down
        gc.collect()
        gc.disable()
        try:
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            P.bkry_bdot_noalloc(h, X, Y, G, kind, q)
            torch.cuda.synchronize()
            after = torch.cuda.memory_allocated()
        finally:
            gc.enable()
        assert after == before
        assert np.array_equal(to_np(G), ref)


def test_noalloc_bdot_repeated_small_after_large(h):
    """Many calls alternating sizes: the hand-off counter is cleared per call."""
    p = 8
    Xl, Yl = to_dev(W.gaussian_block(300_000, p, 1)), to_dev(W.gaussian_block(300_000, p, 2))
    Xs, Ys = to_dev(W.gaussian_block(1_000, p, 3)), to_dev(W.gaussian_block(1_000, p, 4))
    rl, rs = to_np(P.bkry_bdot(h, Xl, Yl)), to_np(P.bkry_bdot(h, Xs, Ys))
    G = torch.empty((p, p), dtype=torch.float64, device=Xl.device)
    say("bdot_noalloc alternating")
    for it in range(6):
        X, Y, r = (Xl, Yl, rl) if it % 2 == 0 else (Xs, Ys, rs)
        P.bkry_bdot_noalloc(h, X, Y, G)
        assert np.array_equal(to_np(G), r)


def test_noalloc_bdot_rejects_bad_arguments(h):
    X = to_dev(W.gaussian_block(100, 8, 1))
    G = torch.empty((8, 8), dtype=torch.float64, device=X.device)
    with pytest.raises(P.BkryError):
        P.bkry_bdot_noalloc(h, X, X, G, "hybrid", 3)
