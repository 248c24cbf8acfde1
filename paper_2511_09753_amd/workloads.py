"""Seeded synthetic SPD test matrices.

This module only builds inputs (sparse matrices, right-hand sides, a fixed
pattern for the loss form).  It holds none of the SPAI method's arithmetic, so
both the HIP path and the CPU oracle can be fed from it.

The paper's own test matrices (SuiteSparse and the authors' custom matrices,
Section 7, Table 3) are not available; these generators stand in for them with
stencil and random-graph SPD matrices whose rows carry 5-9 nonzeros, inside the
3-73 range of Table 3.

Conventions
-----------
* Every matrix is returned as ``scipy.sparse.csr_matrix`` in float64 with sorted
  column indices, no duplicates and no stored zeros.
* Grid unknowns are ordered lexicographically with x fastest.
* Random streams use ``numpy.random.default_rng(1000 * config + stream)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "laplace2d", "aniso2d", "lognormal3d", "geometric_graph", "batch_geometric",
    "grid9", "square_pattern", "loss_m_values", "rhs", "Workload", "workload",
    "seed_for",
]


def seed_for(config: int, stream: int = 0) -> int:
    return 1000 * config + stream


def _finish(A: sp.spmatrix) -> sp.csr_matrix:
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def _grid_ops(N: int) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """Sparse 1-D identity and forward-neighbour shift on N points."""
    I = sp.identity(N, format="csr")
    S = sp.diags([np.ones(N - 1)], [1], shape=(N, N), format="csr")
    return I, S


def laplace2d(N: int) -> sp.csr_matrix:
    """5-point Dirichlet Laplacian on an N x N grid: diagonal 4, neighbours -1."""
    return aniso2d(N, 1.0, 1.0)


def aniso2d(N: int, cx: float = 1.0, cy: float = 0.01) -> sp.csr_matrix:
    """5-point anisotropic diffusion on an N x N grid, Dirichlet boundary.

    Coupling ``cx`` along x (the fast index) and ``cy`` along y; diagonal
    ``2 cx + 2 cy`` on every row (boundary rows keep the full diagonal, which
    is the Dirichlet elimination of the missing neighbours).
    """
    I, S = _grid_ops(N)
    T = S + S.T
    off = cx * sp.kron(I, T) + cy * sp.kron(T, I)
    A = (2.0 * cx + 2.0 * cy) * sp.identity(N * N) - off
    return _finish(A)


def lognormal3d(N: int, seed: int, sigma: float = 1.0) -> sp.csr_matrix:
    """7-point finite-volume diffusion on an N^3 grid.

    Cell coefficients ``kappa = exp(sigma * xi)``, ``xi ~ N(0, 1)`` i.i.d.  An
    interior face between cells c, c' gets the harmonic mean
    ``2 kappa_c kappa_c' / (kappa_c + kappa_c')``; a Dirichlet boundary face of
    cell c gets ``kappa_c``.  Off-diagonals are minus the face coefficient and
    the diagonal is the sum of the cell's face coefficients.
    """
    rng = np.random.default_rng(seed)
    kap = np.exp(sigma * rng.standard_normal((N, N, N)))  # indexed [z, y, x]
    n = N ** 3
    idx = np.arange(n).reshape(N, N, N)
    diag = np.zeros((N, N, N))
    rows, cols, vals = [], [], []
    for axis in (2, 1, 0):  # x, y, z
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, N - 1)
        hi[axis] = slice(1, N)
        ka, kb = kap[tuple(lo)], kap[tuple(hi)]
        face = 2.0 * ka * kb / (ka + kb)
        diag[tuple(lo)] += face
        diag[tuple(hi)] += face
        ia, ib = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        f = face.ravel()
        rows += [ia, ib]
        cols += [ib, ia]
        vals += [-f, -f]
        # Dirichlet faces on both ends of this axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = slice(0, 1)
        last[axis] = slice(N - 1, N)
        diag[tuple(first)] += kap[tuple(first)]
        diag[tuple(last)] += kap[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _finish(A)


def _morton_order(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    qx = np.minimum((x * 65536).astype(np.uint64), 65535)
    qy = np.minimum((y * 65536).astype(np.uint64), 65535)

    def spread(v):
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v

    code = spread(qx) | (spread(qy) << np.uint64(1))
    return np.argsort(code, kind="stable")


def geometric_radius(n: int, mean_degree: float = 8.0) -> float:
    """Radius r with (n-1)(pi r^2 - 8 r^3 / 3 + r^4 / 2) = mean_degree.

    The bracket is the expected number of other uniform points of the unit
    square within distance r of a uniform point (boundary effects included).
    """
    f = lambda r: (n - 1) * (math.pi * r * r - 8.0 * r ** 3 / 3.0 + r ** 4 / 2.0) - mean_degree
    lo, hi = 0.0, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def geometric_graph(n: int, seed: int, shift: float | None = None) -> sp.csr_matrix:
    """Random geometric graph Laplacian (unit weights) plus ``shift * I``.

    Points are uniform in the unit square and ordered by Morton code; edges join
    points closer than ``geometric_radius(n)``.  ``shift`` defaults to a draw from
    U(1e-3, 1e-1) from the same stream.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    if shift is None:
        shift = float(rng.uniform(1e-3, 1e-1))
    pts = pts[_morton_order(pts[:, 0], pts[:, 1])]
    r = geometric_radius(n)
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    W = sp.coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n))
    W = (W + W.T).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    A = sp.diags(deg + shift) - W
    return _finish(A)


def batch_geometric(count: int, seed: int, nmin: int = 500, nmax: int = 20000):
    """``count`` geometric-graph SPD matrices with sizes n ~ U{nmin..nmax}."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    subseeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [geometric_graph(int(s), int(q)) for s, q in zip(sizes, subseeds)]


def grid9(N: int, seed: int, lo: float = 0.5, hi: float = 2.0) -> sp.csr_matrix:
    """8-neighbour grid-graph Laplacian with U(lo, hi) edge weights.

    Each node also gets, for every one of its 8 neighbour directions that leaves
    the grid, a Dirichlet weight U(lo, hi) added to its diagonal.
    """
    rng = np.random.default_rng(seed)
    n = N * N
    idx = np.arange(n).reshape(N, N)  # [y, x]
    rows, cols, vals = [], [], []
    diag = np.zeros((N, N))
    for dy, dx in ((0, 1), (1, 0), (1, 1), (1, -1)):
        # source (y, x) and target (y + dy, x + dx), both inside the grid
        y0 = np.arange(0, N - dy)
        x0 = np.arange(max(0, -dx), N - max(0, dx))
        ys, xs = np.meshgrid(y0, x0, indexing="ij")
        yt, xt = ys + dy, xs + dx
        a = idx[ys, xs]
        b = idx[yt, xt]
        w = rng.uniform(lo, hi, size=a.shape)
        np.add.at(diag, (ys, xs), w)
        np.add.at(diag, (yt, xt), w)
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [-w.ravel(), -w.ravel()]
    # Dirichlet boundary weights: count the outward directions of each node
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    missing = np.zeros((N, N), dtype=np.int64)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            out = (yy + dy < 0) | (yy + dy >= N) | (xx + dx < 0) | (xx + dx >= N)
            missing += out
    bw = rng.uniform(lo, hi, size=(N, N, 8))
    mask = np.arange(8)[None, None, :] < missing[:, :, None]
    diag += (bw * mask).sum(axis=2)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _finish(A)


def square_pattern(A: sp.csr_matrix) -> sp.csr_matrix:
    """Boolean pattern of A^2 (as a float matrix of ones), for the loss form."""
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    Q = (P @ P).tocsr()
    Q.data[:] = 1.0
    return _finish(Q)


def loss_m_values(A: sp.csr_matrix, pattern: sp.csr_matrix, seed: int) -> sp.csr_matrix:
    """Values for the fixed-pattern loss input M.

    Diagonal ``1 / a_jj``; off-diagonal ``0.1 * U(-1, 1) / sqrt(a_kk a_jj)``.
    """
    rng = np.random.default_rng(seed)
    d = A.diagonal()
    Pc = pattern.tocoo()
    r, c = Pc.row, Pc.col
    v = 0.1 * rng.uniform(-1.0, 1.0, size=len(r)) / np.sqrt(d[r] * d[c])
    on = r == c
    v[on] = 1.0 / d[r[on]]
    M = sp.coo_matrix((v, (r, c)), shape=A.shape)
    return _finish(M)


# ----------------------------------------------------------------------------
# The paper's own custom matrices, rebuilt from their recipes (Section 7, the list of
# test matrices and Table 3).  The draws are seeded here, so each realisation differs
# from the authors'; structure, value ranges and nnz follow the recipes.
# Readings: "eigenvalues of L" are its diagonal entries (L is triangular); the 100 random
# diagonal entries are the first 100 (one contiguous run: scattered at random positions
# they leave tri100eigs4k with lambda_min near 1e-3, far from the near-singularity of
# 1e-8 the paper states, while the leading run gives 1e-7 .. 1e-8, and 1e-9 for
# 4bw100eigs20k, as Table 3 reports); "dense
# bandwidth of 4" means four full sub-diagonals (nnz(A) = 9n - 20, as in Table 3);
# rand20k's L has one sub-diagonal entry per row i >= 1, in a column drawn uniformly
# from 0 .. i-1 (nnz(A) then comes within a percent of Table 3's 99,772); rand20k2
# shares rand20k's pattern and off-diagonal values.
# ----------------------------------------------------------------------------

PAPER_RECIPES = ("tri100eigs4k", "4bw100eigs20k", "4bw100eigs20k2", "rand20k", "rand20k2")


def _llt(L: sp.spmatrix) -> sp.csr_matrix:
    """A = L L^T, made exactly (bitwise) symmetric."""
    L = sp.csr_matrix(L)
    A = sp.csr_matrix(L @ L.T)
    return _finish(0.5 * (A + A.T))


def _random_diagonal(n: int, count: int, lo: float, hi: float, rng) -> np.ndarray:
    d = np.ones(n)
    d[:count] = rng.uniform(lo, hi, size=count)
    return d


def paper_recipe(name: str, seed: int) -> sp.csr_matrix:
    """One of the paper's custom test matrices (tri100eigs4k, 4bw100eigs20k,
    4bw100eigs20k2, rand20k, rand20k2), A = L L^T as its recipe describes."""
    rng = np.random.default_rng(seed)
    if name == "tri100eigs4k":
        n = 4000
        d = _random_diagonal(n, 100, 0.05, 1.05, rng)
        sub = rng.uniform(0.0, 1.0, size=n - 1)
        return _llt(sp.diags([d, sub], [0, -1]))
    if name in ("4bw100eigs20k", "4bw100eigs20k2"):
        n = 20000
        hi = 0.05 if name == "4bw100eigs20k" else 1e5
        d = _random_diagonal(n, 100, 0.0, hi, rng)
        subs = [rng.uniform(0.0, 0.01, size=n - k) for k in range(1, 5)]
        return _llt(sp.diags([d] + subs, [0, -1, -2, -3, -4]))
    if name in ("rand20k", "rand20k2"):
        n = 20000
        prng = np.random.default_rng(seed)          # pattern and off-diagonal values shared
        rows = np.arange(1, n)
        cols = (prng.random(n - 1) * rows).astype(np.int64)
        vals = prng.uniform(0.0, 1.0, size=n - 1)
        hi = 1e4 if name == "rand20k" else 1e2
        d = np.random.default_rng(seed + 1).uniform(0.0, hi, size=n)
        L = sp.coo_matrix((np.concatenate([d, vals]),
                           (np.concatenate([np.arange(n), rows]), np.concatenate([np.arange(n), cols]))),
                          shape=(n, n))
        return _llt(L)
    raise ValueError(f"unknown recipe {name}")


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides b ~ U(-1, 1), shape (n, nrhs), row-major (RHS fastest)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(n, nrhs)))


@dataclass
class Workload:
    """A named configuration: matrices plus the iteration recipe."""
    name: str
    A: object                       # csr_matrix, or list of them (batched)
    method: str                     # "mr" | "cg" | "lomr"
    cap_mode: str                   # "none" | "global" | "column"
    cap_value: float                # global: absolute m; column: factor x nnz(A e_j), or absolute k
    cap_relative: bool
    iters: int
    nrhs: int
    rtol: float = 1e-8
    precision: str = "f64"
    extra: dict = field(default_factory=dict)


def workload(name: str, small: bool = False) -> Workload:
    """The five synthetic configurations (and reduced variants for tests).

    * ``laplace32``   2D 5-point Laplacian 32x32, MR, global cap nnz(A), 20 its, 1 RHS.
    * ``aniso256``    2D anisotropic 256x256 (ratio 100), per-column cap 3 nnz(A e_j),
                      50 its of MR / LOMR / CG, 4 RHS.
    * ``lognormal96`` 3D 7-point lognormal 96^3, LOMR FP32 values, global cap 2 nnz(A),
                      30 its, 64 RHS.
    * ``geo256``      256 geometric-graph Laplacians n ~ U{500..20000}, MR, column cap 4,
                      20 its, FP32 values.
    * ``grid9_512``   9-point grid graph 512x512, loss on pattern(A^2).
    """
    if name == "laplace32":
        N = 8 if small else 32
        A = laplace2d(N)
        return Workload(name, A, "mr", "global", float(A.nnz), False, 20, 1)
    if name == "aniso256":
        N = 32 if small else 256
        A = aniso2d(N, 1.0, 0.01)
        return Workload(name, A, "lomr", "column", 3.0, True, 50, 4)
    if name == "lognormal96":
        N = 16 if small else 96
        A = lognormal3d(N, seed_for(3))
        return Workload(name, A, "lomr", "global", 2.0 * A.nnz, False, 30, 64, precision="f32")
    if name == "geo256":
        count, nmax = (8, 2000) if small else (256, 20000)
        As = batch_geometric(count, seed_for(4), 500, nmax)
        return Workload(name, As, "mr", "column", 4.0, False, 20, 1, precision="f32")
    if name == "grid9_512":
        N = 32 if small else 512
        A = grid9(N, seed_for(5))
        return Workload(name, A, "mr", "none", 0.0, False, 0, 0, precision="f32",
                        extra={"pattern": square_pattern(A)})
    raise KeyError(name)
