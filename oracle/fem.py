"""Bilinear (Q1) finite elements for the anisotropic diffusion of Example 1
(Sec. 3): -div(K grad u) = f on (0,1)^2 with K = diag(kxx, kyy) (eq. (1)),
on a uniform mesh of m x m square elements (FP64 oracle, test
infrastructure only).

Readings (listed in DESIGN): the element type is unstated, bilinear Q1 on
squares is taken; boundary conditions and right-hand side are unstated,
homogeneous Dirichlet on the whole boundary and f = 1 are taken.  The
unknowns are the (m-1)^2 interior nodes, x fastest, so that the level
hierarchy of ``oracle.hierarchy`` (coarse node J on fine node 2J+1) is the
nested mesh hierarchy of uniform refinement.

The element matrix is integrated with the 2 x 2 Gauss rule, exact for the
bilinear basis: K_e[a, b] = sum_q w_q (kxx dphi_a/dx dphi_b/dx +
kyy dphi_a/dy dphi_b/dy) |J|.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _element_matrix(h: float, kxx: float, kyy: float) -> np.ndarray:
    """4 x 4 stiffness of one square element, local nodes (0,0), (1,0),
    (0,1), (1,1) (x fastest), by 2 x 2 Gauss quadrature."""
    g = 1.0 / math.sqrt(3.0)
    pts = [(-g, -g), (g, -g), (-g, g), (g, g)]
    corners = [(-1, -1), (1, -1), (-1, 1), (1, 1)]
    Ke = np.zeros((4, 4))
    for (xi, eta) in pts:
        # bilinear basis on the reference square [-1, 1]^2
        dxi = np.array([c[0] * (1 + c[1] * eta) / 4.0 for c in corners])
        deta = np.array([c[1] * (1 + c[0] * xi) / 4.0 for c in corners])
        dx = dxi * (2.0 / h)           # d/dx = (2/h) d/dxi
        dy = deta * (2.0 / h)
        jac = (h / 2.0) ** 2
        Ke += (kxx * np.outer(dx, dx) + kyy * np.outer(dy, dy)) * jac   # unit Gauss weights
    return Ke


def stiffness(m: int, kxx: float, kyy: float = 1.0) -> sp.csr_matrix:
    """Assembled stiffness on the (m-1)^2 interior nodes (Dirichlet rows and
    columns of the boundary nodes removed)."""
    h = 1.0 / m
    Ke = _element_matrix(h, kxx, kyy)
    n = m - 1                                   # interior nodes per axis
    rows, cols, vals = [], [], []

    def gid(ix, iy):                            # global node (0..m) -> interior index or -1
        if ix <= 0 or iy <= 0 or ix >= m or iy >= m:
            return -1
        return (ix - 1) + n * (iy - 1)

    for ey in range(m):
        for ex in range(m):
            nodes = [gid(ex, ey), gid(ex + 1, ey), gid(ex, ey + 1), gid(ex + 1, ey + 1)]
            for a in range(4):
                if nodes[a] < 0:
                    continue
                for b in range(4):
                    if nodes[b] < 0:
                        continue
                    rows.append(nodes[a])
                    cols.append(nodes[b])
                    vals.append(Ke[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def load(m: int, f: float = 1.0) -> np.ndarray:
    """Consistent load vector of a constant f: int f phi_i = f h^2 per interior node."""
    h = 1.0 / m
    return np.full((m - 1) ** 2, f * h * h)


def stencil(m: int, kxx: float, kyy: float = 1.0) -> np.ndarray:
    """The 3 x 3 interior stencil (rows dy = -1, 0, 1; columns dx = -1, 0, 1)
    read off the assembled matrix at an interior node."""
    A = stiffness(m, kxx, kyy).tocsr()
    n = m - 1
    c = (n // 2) + n * (n // 2)
    st = np.zeros((3, 3))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            st[dy + 1, dx + 1] = A[c, c + dx + n * dy]
    return st
