"""The nested hierarchy V_0 c V_1 c ... c V_L of Sec. 2.1 (FP64 oracle).

Level L is the finest (the given A); level l < L has Galerkin operator
A_l = R_l A_{l+1} P_l with P_l the tensor linear interpolation from level l to
level l+1 and R_l = 2^{-d} P_l^T.  Composite transfers P_l^L are applied as
products of these two-level operators (Sec. 2.1 allows composite or explicit
operators; both implementations here use the composite form).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import operators as ops


class NotSPDError(ValueError):
    """A level operator has a non-positive diagonal entry."""


@dataclass
class Level:
    n: int                       # nodes per axis
    A: sp.csr_matrix             # level operator A_l
    D: np.ndarray                # its diagonal
    P: Optional[sp.csr_matrix]   # interpolation to the next finer level (None at L)
    R: Optional[sp.csr_matrix]   # restriction from the next finer level (None at L)


@dataclass
class Hierarchy:
    dim: int
    levels: List[Level]          # index 0 = coarsest, -1 = finest

    @property
    def L(self) -> int:
        return len(self.levels) - 1

    @property
    def fine(self) -> Level:
        return self.levels[-1]


def build(dim: int, n: int, nlevels: int, A: sp.spmatrix | None = None,
          kappa: np.ndarray | None = None) -> Hierarchy:
    """Build ``nlevels`` levels below and including the fine FD operator."""
    if A is None:
        A = ops.fd_matrix(dim, n, kappa)
    A = sp.csr_matrix(A, dtype=np.float64)
    sizes = [n]
    for _ in range(nlevels - 1):
        sizes.append(sizes[-1] // 2)
    if sizes[-1] < 1:
        raise ValueError("too many levels for this grid")
    finest_first = [Level(n, A, A.diagonal().copy(), None, None)]
    for l in range(1, nlevels):
        nf = sizes[l - 1]
        P = ops.prolongation(dim, nf)
        R = ops.restriction(dim, nf)
        Af = finest_first[-1].A
        Ac = ops.galerkin(Af, P, R)
        lev = Level(sizes[l], Ac, Ac.diagonal().copy(), P, R)
        finest_first.append(lev)
    levels = finest_first[::-1]
    # P/R stored on level l describe the transfer to/from level l+1
    for lev in levels:
        if np.any(~(lev.D > 0.0)):
            raise NotSPDError("non-positive diagonal in a level operator")
    return Hierarchy(dim, levels)


def restrict_to(h: Hierarchy, r: np.ndarray, l: int) -> np.ndarray:
    """R_L^l r by successive two-level restrictions (identity at l = L)."""
    g = r
    for j in range(h.L - 1, l - 1, -1):
        g = h.levels[j].R @ g
    return g


def prolong_from(h: Hierarchy, c: np.ndarray, l: int) -> np.ndarray:
    """P_l^L c by successive two-level interpolations (identity at l = L)."""
    z = c
    for j in range(l, h.L):
        z = h.levels[j].P @ z
    return z


def from_operators(A: sp.spmatrix, prolongations, restrict_scale: float) -> Hierarchy:
    """A level hierarchy from a fine matrix and given prolongations (Sec. 2.1
    for a general nested hierarchy): prolongations[l] maps level l to level
    l+1 (level 0 coarsest), R_l = restrict_scale * P_l^T and the coarse
    operators are the Galerkin products R A P (stored symmetrised).  The
    ``n`` of a level is its number of unknowns."""
    A = sp.csr_matrix(A, dtype=np.float64)
    Ps = [sp.csr_matrix(P, dtype=np.float64) for P in prolongations]
    finest_first = [Level(A.shape[0], A, A.diagonal().copy(), None, None)]
    for P in reversed(Ps):
        Af = finest_first[-1].A
        if P.shape[0] != Af.shape[0]:
            raise ValueError("prolongation rows must match the finer level")
        R = (restrict_scale * P.T).tocsr()
        Ac = ops.galerkin(Af, P, R)
        finest_first.append(Level(P.shape[1], Ac, Ac.diagonal().copy(), P, R))
    levels = finest_first[::-1]
    for lev in levels:
        if np.any(~(lev.D > 0.0)):
            raise NotSPDError("non-positive diagonal in a level operator")
    return Hierarchy(0, levels)
