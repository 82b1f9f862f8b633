"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module builds matrices and right-hand sides only; it holds none of the
block Krylov arithmetic.  The paper's own experiments use SuiteSparse
matrices that are not available here, so stencil matrices of the kinds the
paper itself uses for its kernel benchmarks (finite-difference Poisson
problems, Ch. 3 "Numerical Experiments") stand in for them, at the sizes of
the workload table below.

Conventions for every grid matrix:
  * unknowns are the interior nodes of a uniform grid (Dirichlet boundary
    nodes eliminated), ordered lexicographically with x fastest;
  * CSR with 0-based int32 indices and columns sorted inside each row;
  * values are float64.
Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np


@dataclasses.dataclass
class Csr:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.val
        return d


def _stencil_csr(shape, offsets, weight_fn):
    """Assemble a stencil matrix on the interior grid ``shape`` (x fastest).

    ``offsets`` is a list of integer displacement tuples (dx, dy[, dz]).
    ``weight_fn(off, valid)`` returns the value array (one entry per grid node)
    for that displacement.  Entries whose neighbour lies outside the grid are
    dropped (eliminated Dirichlet nodes).
    """
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [1]
    for d in shape[:-1]:
        strides.append(strides[-1] * d)
    # sort displacements by linear offset so that columns come out sorted
    offsets = sorted(offsets, key=lambda o: sum(o[k] * strides[k] for k in range(dims)))
    coords = np.indices(shape[::-1]).reshape(dims, -1)[::-1]  # coords[k] varies as axis k, x fastest
    lin = np.arange(n, dtype=np.int64)
    cols = np.empty((n, len(offsets)), dtype=np.int64)
    vals = np.empty((n, len(offsets)), dtype=np.float64)
    for j, off in enumerate(offsets):
        valid = np.ones(n, dtype=bool)
        for k in range(dims):
            c = coords[k] + off[k]
            valid &= (c >= 0) & (c < shape[k])
        cols[:, j] = np.where(valid, lin + sum(off[k] * strides[k] for k in range(dims)), -1)
        vals[:, j] = weight_fn(off, valid)
    keep = cols >= 0
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[keep].astype(np.int32)
    val = vals[keep]
    assert rowptr[-1] < 2**31
    return Csr(n, rowptr.astype(np.int32), colind, val)


def laplace_2d(N: int) -> Csr:
    """5-point Laplacian [-1; -1 4 -1; -1] on an N x N interior grid (unscaled)."""
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]

    def w(off, valid):
        return np.full(valid.shape, 4.0 if off == (0, 0) else -1.0)

    return _stencil_csr((N, N), offs, w)


def laplace_3d(N: int) -> Csr:
    """7-point Laplacian (diagonal 6, neighbours -1) on an N^3 interior grid."""
    offs = [(0, 0, 0)] + [tuple(int(i == k) * sgn for i in range(3)) for k in range(3) for sgn in (1, -1)]

    def w(off, valid):
        return np.full(valid.shape, 6.0 if off == (0, 0, 0) else -1.0)

    return _stencil_csr((N, N, N), offs, w)


def _lognormal_nodes(N: int, dims: int, sigma: float, seed: int) -> np.ndarray:
    """Node coefficients exp(sigma * xi), xi ~ N(0,1) iid, on the grid extended
    by one boundary layer, shape (N+2,)*dims indexed [z][y][x] (x fastest)."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((N + 2,) * dims)
    return np.exp(sigma * xi)


def _variable_diffusion(N: int, sigma: float, seed: int, max_l1: int) -> Csr:
    """Weighted graph Laplacian over the neighbours with |d|_inf = 1 and
    |d|_1 <= max_l1 (1: 7-point, 3: 27-point).  Edge weight between nodes i, j is
    omega_d * harmonic mean 2 k_i k_j / (k_i + k_j), omega = 1, 1/2, 1/3 for
    face, edge and corner neighbours; a_ij = -w_ij and a_ii = sum of w_ij over
    all neighbours, including eliminated boundary nodes, so A is SPD."""
    kap = _lognormal_nodes(N, 3, sigma, seed)
    ki = kap[1:-1, 1:-1, 1:-1].reshape(-1)
    nbr = [d for d in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(map(abs, d)) <= max_l1]
    omega = {1: 1.0, 2: 0.5, 3: 1.0 / 3.0}

    def edge_w(d):
        dx, dy, dz = d
        kj = kap[1 + dz:N + 1 + dz, 1 + dy:N + 1 + dy, 1 + dx:N + 1 + dx].reshape(-1)
        return omega[abs(dx) + abs(dy) + abs(dz)] * 2.0 * ki * kj / (ki + kj)

    diag = np.zeros(N ** 3)
    for d in nbr:
        diag += edge_w(d)

    def w(off, valid):
        if off == (0, 0, 0):
            return diag
        return -edge_w(off)

    return _stencil_csr((N, N, N), [(0, 0, 0)] + nbr, w)


def diffusion_27pt(N: int, sigma: float = 1.0, seed: int = 1003) -> Csr:
    """27-point variable-coefficient diffusion with log-normal node coefficients."""
    return _variable_diffusion(N, sigma, seed, 3)


def diffusion_7pt_var(N: int, sigma: float = 1.0, seed: int = 1005) -> Csr:
    """7-point variable-coefficient diffusion; face coefficients are harmonic
    means of log-normal node coefficients."""
    return _variable_diffusion(N, sigma, seed, 1)


def convdiff_2d(N: int, wind=(1.0, 0.5), pe_h: float = 10.0) -> Csr:
    """First-order upwind discretisation of -eps*Lap(u) + w.grad(u) on the unit
    square with h = 1/(N+1), scaled by h^2/eps, at cell Peclet number
    Pe_h = |w|_2 h / (2 eps).  Nonsymmetric M-matrix."""
    wx, wy = wind
    wn = math.hypot(wx, wy)
    cx = 2.0 * pe_h * abs(wx) / wn
    cy = 2.0 * pe_h * abs(wy) / wn
    up_x = (-1, 0) if wx >= 0 else (1, 0)
    up_y = (0, -1) if wy >= 0 else (0, 1)
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]

    def w(off, valid):
        if off == (0, 0):
            v = 4.0 + cx + cy
        elif off == up_x:
            v = -1.0 - cx
        elif off == up_y:
            v = -1.0 - cy
        else:
            v = -1.0
        return np.full(valid.shape, v)

    return _stencil_csr((N, N), offs, w)


def uniform_block(n: int, s: int, seed: int) -> np.ndarray:
    """n x s row-major block with entries uniform in [-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, s))


def gaussian_block(n: int, s: int, seed: int) -> np.ndarray:
    """n x s row-major block with standard normal entries."""
    return np.random.default_rng(seed).standard_normal((n, s))


def color_priorities(n: int, seed: int) -> np.ndarray:
    """Uniform uint32 priorities for the multicolour ordering (one per row)."""
    return np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint32)


def random_spd_csr(n: int, density: float, seed: int, shift: float = 1.0) -> Csr:
    """Small random sparse SPD matrix (symmetric pattern, diagonally dominant),
    for tests over shapes that are not grids.  Integer-valued off-diagonals."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    mask = np.triu(mask, 1)
    vals = np.where(mask, -rng.integers(1, 4, size=(n, n)).astype(np.float64), 0.0)
    a = vals + vals.T
    a[np.diag_indices(n)] = -a.sum(axis=1) + shift
    return dense_to_csr(a)


def random_csr(n: int, m_cols: int, density: float, seed: int, integer: bool = True,
               empty_rows=()) -> Csr:
    """Random rectangular-pattern CSR (n rows, columns < m_cols); optional empty rows."""
    rng = np.random.default_rng(seed)
    d = np.where(rng.random((n, m_cols)) < density,
                 rng.integers(-4, 5, size=(n, m_cols)).astype(np.float64) if integer
                 else rng.standard_normal((n, m_cols)), 0.0)
    for r in empty_rows:
        d[r, :] = 0.0
    return dense_to_csr(d, square=False)


def dense_to_csr(a: np.ndarray, square: bool = True) -> Csr:
    """CSR of the non-zero entries of a dense matrix (sorted columns)."""
    if square:
        assert a.shape[0] == a.shape[1]
    nz = a != 0.0
    rowptr = np.zeros(a.shape[0] + 1, dtype=np.int32)
    np.cumsum(nz.sum(axis=1), out=rowptr[1:])
    r, c = np.nonzero(nz)
    return Csr(a.shape[0], rowptr, c.astype(np.int32), a[r, c].astype(np.float64))


# ---------------------------------------------------------------------------
# The five workloads.  Each entry states the matrix, the block of right-hand
# sides and the seed.  ``build_workload(name)`` returns (A, B, extra).
# ---------------------------------------------------------------------------
WORKLOADS = {
    "poisson2d_32x32_s4": dict(matrix=("laplace_2d", 32), rhs=("uniform", 4, 1001)),
    "laplace3d_128_s8": dict(matrix=("laplace_3d", 128), rhs=("uniform", 8, 1002)),
    "diffusion27_96_s16": dict(matrix=("diffusion_27pt", 96, 1.0, 1003), rhs=("gaussian", 16, 2003)),
    "convdiff2d_1024_s8": dict(matrix=("convdiff_2d", 1024), rhs=("gaussian", 8, 1004)),
    "diffusion7var_64_s32": dict(matrix=("diffusion_7pt_var", 64, 1.0, 1005), rhs=("gaussian", 32, 2005),
                                 target=("gaussian", 32, 3005)),
}

_MATRIX_FNS = {
    "laplace_2d": laplace_2d,
    "laplace_3d": laplace_3d,
    "diffusion_27pt": diffusion_27pt,
    "diffusion_7pt_var": diffusion_7pt_var,
    "convdiff_2d": convdiff_2d,
}


def build_matrix(spec) -> Csr:
    fn = _MATRIX_FNS[spec[0]]
    return fn(*spec[1:])


def build_block(spec, n: int) -> np.ndarray:
    kind, s, seed = spec
    return uniform_block(n, s, seed) if kind == "uniform" else gaussian_block(n, s, seed)


def build_workload(name: str, grid: int | None = None):
    """Build a named workload.  ``grid`` optionally replaces the grid size
    (same generator, same seeds) for reduced-size runs."""
    w = WORKLOADS[name]
    mspec = list(w["matrix"])
    if grid is not None:
        mspec[1] = grid
    A = build_matrix(mspec)
    B = build_block(w["rhs"], A.n)
    extra = {}
    if "target" in w:
        extra["target"] = build_block(w["target"], A.n)
    return A, B, extra


TSQR_WORKLOAD = dict(m=4_194_304, c=32, seed=1044)


def tsqr_input(m: int = TSQR_WORKLOAD["m"], c: int = TSQR_WORKLOAD["c"], seed: int = TSQR_WORKLOAD["seed"]):
    """Gaussian m x c matrix for the standalone tall-skinny QR workload."""
    return gaussian_block(m, c, seed)
