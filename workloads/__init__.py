"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws numbers and describes problem shapes.  It holds none of
the solver's arithmetic (no operators, no transfers, no smoothing, no Krylov
steps), so the oracle and the HIP path can both take their inputs from here
without sharing any of the method.

Workloads (all synthetic; the paper's own experiments use FEM meshes and a
fracture geometry that are not reproduced here):

* ``poisson2d_31``   2D, 31x31 interior nodes, 4 levels (31/15/7/3), b ~ U[-1,1], seed 1.
* ``poisson3d_127``  3D, 127^3 interior nodes, 6 levels (127/63/31/15/7/3), b ~ U[-1,1], seed 2.
* ``diffusion3d_127`` as above with kappa = exp(2 g), g a unit-variance Gaussian
  field with squared-exponential covariance, correlation length 1/16, seed 3.
* ``batched2d_512``  512 independent 2D Poisson instances, side n_i ~ U{31..255}
  (seed 4), rhs seed 4000+i, levels max(2, floor(log2(n_i+1)) - 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass(frozen=True)
class GridProblem:
    """A structured problem: ``dim``-D unit cube, ``n`` interior nodes per axis."""
    name: str
    dim: int
    n: int
    nlevels: int
    rhs_seed: int
    kappa_seed: Optional[int] = None   # None => kappa == 1 (Poisson)
    corr_len: float = 1.0 / 16.0

    @property
    def ndof(self) -> int:
        return self.n ** self.dim


POISSON2D_31 = GridProblem("poisson2d_31", 2, 31, 4, rhs_seed=1)
POISSON3D_127 = GridProblem("poisson3d_127", 3, 127, 6, rhs_seed=2)
DIFFUSION3D_127 = GridProblem("diffusion3d_127", 3, 127, 6, rhs_seed=2, kappa_seed=3)
# beyond the 256 MB Infinity Cache: 16,581,375 DoF, 7 levels (255 .. 3)
POISSON3D_255 = GridProblem("poisson3d_255", 3, 255, 7, rhs_seed=2)

PROBLEMS = {p.name: p for p in (POISSON2D_31, POISSON3D_127, DIFFUSION3D_127)}


def level_sizes(n: int, nlevels: int) -> List[int]:
    """Per-axis node counts, finest first: n, floor(n/2), floor(n/4), ..."""
    sizes = [n]
    for _ in range(nlevels - 1):
        sizes.append(sizes[-1] // 2)
    if sizes[-1] < 1:
        raise ValueError(f"n={n} too small for {nlevels} levels")
    return sizes


def rhs(ndof: int, seed: int) -> np.ndarray:
    """b ~ U[-1, 1]^ndof in float64 from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=ndof)


def gaussian_field(n: int, dim: int, seed: int, corr_len: float = 1.0 / 16.0,
                   periodic: int = 256, workers: Optional[int] = None) -> np.ndarray:
    """Unit-variance stationary Gaussian field on the (n+2)^dim node grid.

    Covariance exp(-r^2 / (2 corr_len^2)) with node spacing h = 1/(n+1),
    synthesised by circulant embedding on a periodic ``periodic``^dim grid of
    the same spacing and cropped to the (n+2)^dim corner (boundary nodes
    included).  Returned with x fastest: shape (n+2,)*dim indexed [z, y, x].
    ``workers``: use scipy's multi-threaded FFT (same field up to rounding;
    for bulk generation of training fields).  Default: numpy's FFT.
    """
    m = periodic
    if m < n + 2:
        raise ValueError("periodic grid smaller than the node grid")
    h = 1.0 / (n + 1)
    d1 = np.minimum(np.arange(m), m - np.arange(m)) * h  # periodic distance
    r2 = np.zeros((m,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = m
        r2 = r2 + (d1 ** 2).reshape(shape)
    cov = np.exp(-r2 / (2.0 * corr_len ** 2))
    if workers is None:
        fftn, ifftn = np.fft.fftn, np.fft.ifftn
    else:
        import scipy.fft as sfft
        fftn = lambda a: sfft.fftn(a, workers=workers)
        ifftn = lambda a: sfft.ifftn(a, workers=workers)
    spec = np.real(fftn(cov))
    spec = np.maximum(spec, 0.0)
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((m,) * dim)
    g = np.real(ifftn(np.sqrt(spec) * fftn(white)))
    crop = tuple(slice(0, n + 2) for _ in range(dim))
    return np.ascontiguousarray(g[crop])


def kappa_field(problem: GridProblem, workers: Optional[int] = None) -> Optional[np.ndarray]:
    """kappa = exp(2 g) on the (n+2)^dim node grid, or None for Poisson."""
    if problem.kappa_seed is None:
        return None
    g = gaussian_field(problem.n, problem.dim, problem.kappa_seed, problem.corr_len, workers=workers)
    return np.exp(2.0 * g)


# Learned direction on the heterogeneous 127^3 problem: training kappa seeds
# 10000 + j, held-out test seeds 900000 + i (rhs seed = kappa seed + 1).
TRAIN_KAPPA_SEED0 = 10000
TEST_KAPPA_SEED0 = 900000


def diffusion_instance(kappa_seed: int, n: int = 127, nlevels: int = 6) -> GridProblem:
    """A fresh heterogeneous instance from the distribution of diffusion3d_127."""
    return GridProblem(f"diffusion3d_{n}_k{kappa_seed}", 3, n, nlevels, rhs_seed=kappa_seed + 1,
                       kappa_seed=kappa_seed)


def problem_rhs(problem: GridProblem) -> np.ndarray:
    return rhs(problem.ndof, problem.rhs_seed)


@dataclass(frozen=True)
class BatchedInstance:
    index: int
    n: int
    nlevels: int
    rhs_seed: int

    @property
    def ndof(self) -> int:
        return self.n * self.n


def batched_levels(n: int) -> int:
    """Hierarchy depth for an instance of side n: max(2, floor(log2(n+1)) - 2)."""
    return max(2, int(math.floor(math.log2(n + 1))) - 2)


def batched_instances(count: int = 512, seed: int = 4, nmin: int = 31,
                      nmax: int = 255) -> List[BatchedInstance]:
    """``count`` 2D Poisson instances with side n_i ~ U{nmin..nmax} (seed)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(nmin, nmax + 1, size=count)
    return [BatchedInstance(i, int(s), batched_levels(int(s)), 4000 + i)
            for i, s in enumerate(sides)]


def batched_rhs(inst: BatchedInstance) -> np.ndarray:
    return rhs(inst.ndof, inst.rhs_seed)


def manufactured_rhs(dim: int, n: int) -> np.ndarray:
    """f = dim * pi^2 * prod_i sin(pi x_i) at interior nodes (x fastest).

    The continuous solution of -Laplace(u) = f with u = 0 on the boundary is
    u = prod_i sin(pi x_i); see ``manufactured_solution``.
    """
    return dim * math.pi ** 2 * manufactured_solution(dim, n)


def manufactured_solution(dim: int, n: int) -> np.ndarray:
    h = 1.0 / (n + 1)
    s = np.sin(math.pi * h * np.arange(1, n + 1))
    u = s
    for _ in range(dim - 1):
        u = np.multiply.outer(s, u)
    return u.reshape(-1).copy()


# ---------------------------------------------------------------- Example 1
# Anisotropic diffusion -div(diag(kxx, kyy) grad u) = f on (0,1)^2 (Sec. 3,
# Example 1): 160 x 160 bilinear elements, 4 nested levels (coarsest
# 20 x 20 elements), kxx in 10^-7 .. 1, kyy = 1.  Unstated in the paper and
# taken here: homogeneous Dirichlet on the whole boundary, f = 1.

EXAMPLE1_ELEMENTS = 160
EXAMPLE1_LEVELS = 4
EXAMPLE1_KXX = [10.0 ** e for e in range(-7, 1)]


def example1_stencil(kxx: float, kyy: float = 1.0) -> np.ndarray:
    """Interior 9-point stencil of the assembled bilinear stiffness on square
    elements (rows dy = -1, 0, 1; columns dx = -1, 0, 1): the x part is kxx
    times the 1D stiffness in x tensor the 1D mass in y (h cancels in 2D),
    the y part likewise."""
    stiff = np.array([-1.0, 2.0, -1.0])           # 1D stiffness, times 1/h
    mass = np.array([1.0, 4.0, 1.0]) / 6.0          # 1D mass, times h
    return kxx * np.outer(mass, stiff) + kyy * np.outer(stiff, mass)


def example1_rhs(elements: int = EXAMPLE1_ELEMENTS, f: float = 1.0) -> np.ndarray:
    """Load vector of a constant f on the interior nodes: f h^2 each."""
    h = 1.0 / elements
    return np.full((elements - 1) ** 2, f * h * h)


# ------------------------------------------------------ unstructured graph
# A general sparse SPD problem for the CSR entry point: random points in
# the unit square, the symmetric k-nearest-neighbour graph with weights
# 1 / distance^2, A = diag(degree) - W + shift I (shift = 1e-3 x mean degree),
# and a nested hierarchy of aggregates given by square cells (4 x 4 cells on
# the coarsest level, twice as many per axis on each finer one; empty cells
# dropped), prolongations piecewise constant (restrict_scale 1).


def graph_problem(npts: int = 20000, seed: int = 7, nlevels: int = 4, k: int = 6):
    """(A, prolongations coarsest first, b) as scipy.sparse CSR matrices."""
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((npts, 2))
    dist, nbr = cKDTree(pts).query(pts, k + 1)
    rows = np.repeat(np.arange(npts), k)
    cols = nbr[:, 1:].reshape(-1)
    w = 1.0 / (dist[:, 1:].reshape(-1) ** 2)
    W = sp.csr_matrix((w, (rows, cols)), shape=(npts, npts))
    W = W.maximum(W.T).tocsr()
    deg = np.asarray(W.sum(axis=1)).reshape(-1)
    A = (sp.diags(deg + 1e-3 * deg.mean()) - W).tocsr()
    A.sort_indices()
    # cell index of every point at each coarse level, coarsest first
    cells = []
    for l in range(nlevels - 1):
        g = 4 * 2 ** l
        ij = np.minimum((pts * g).astype(np.int64), g - 1)
        cells.append(ij[:, 0] + g * ij[:, 1])
    Ps = []
    # renumber the non-empty cells of each level; a fine unknown (point or
    # cell) belongs to the cell of the next coarser level containing it
    ids = []
    for l in range(nlevels - 1):
        uniq, inv = np.unique(cells[l], return_inverse=True)
        ids.append((uniq, inv))
    for l in range(nlevels - 1):
        nc = ids[l][0].size
        if l + 1 < nlevels - 1:
            # level l+1 cells -> level l cells, through any point of each finer cell
            uniq_f, inv_f = ids[l + 1]
            first = np.zeros(uniq_f.size, dtype=np.int64)
            first[inv_f[::-1]] = np.arange(npts)[::-1]
            parent = ids[l][1][first]
            nf = uniq_f.size
        else:
            parent = ids[l][1]
            nf = npts
        Ps.append(sp.csr_matrix((np.ones(nf), (np.arange(nf), parent)), shape=(nf, nc)))
    b = rhs(npts, seed + 1)
    return A, Ps, b
