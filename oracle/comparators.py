"""The comparison methods of Sec. 3 (FP64 oracle, test infrastructure only).

Sec. 3 compares additive-MG MPCG with CG preconditioned by the additive MG
method and with CG preconditioned by the (multiplicative) MG V-cycle, with
the work per level matched: the multiplicative method smooths nu_pre times
before and nu_post times after the coarse correction, the additive one
nu = nu_pre + nu_post times.

  additive MG-PCG    B r = sum_l P_l^L S_l^nu R_L^l r  (eq. (3) summed: the
                     row sum of the MPCG block of Algorithm 1)
  MG(V)-PCG          B r = one V-cycle from c = 0 (Sec. 2.1: smoothing on the
                     way from the finest to the coarsest level, then on the
                     way back), with the same transfers and damped-Jacobi
                     smoother as the additive levels

Readings (listed in DESIGN): the paper's smoother (SSOR) is replaced by the
damped Jacobi of the additive levels; the coarsest level of the V-cycle gets
nu_pre + nu_post sweeps from zero (the additive method's coarsest work);
nu_pre = nu_post so that B is symmetric; the outer iteration is textbook PCG
(``oracle.pcg``).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .hierarchy import Hierarchy
from .mpcg import mg_block
from .pcg import pcg
from .smoother import jacobi


def additive_precond(h: Hierarchy, r: np.ndarray, nu: int = 2, omega: float = 2.0 / 3.0) -> np.ndarray:
    """Sum of the L+1 level corrections (eq. (3))."""
    return mg_block(h, r, nu, omega).sum(axis=1)


def vcycle(h: Hierarchy, r: np.ndarray, nu_pre: int = 1, nu_post: int = 1,
           omega: float = 2.0 / 3.0) -> np.ndarray:
    """One V-cycle for A c = r from c = 0, finest level first."""

    def cycle(l: int, g: np.ndarray) -> np.ndarray:
        lev = h.levels[l]
        if l == 0:
            return jacobi(lev.A, lev.D, g, nu_pre + nu_post, omega)
        c = jacobi(lev.A, lev.D, g, nu_pre, omega)                 # pre-smoothing from 0
        coarse = h.levels[l - 1]
        gc = coarse.R @ (g - lev.A @ c)                            # restricted residual
        c = c + coarse.P @ cycle(l - 1, gc)                        # coarse-grid correction
        for _ in range(nu_post):                                   # post-smoothing
            c = c + omega * ((g - lev.A @ c) / lev.D)
        return c

    return cycle(h.L, r)


def additive_pcg(h: Hierarchy, b: np.ndarray, tol: float = 1e-8, maxit: int = 1000, nu: int = 2,
                 omega: float = 2.0 / 3.0, x0: np.ndarray | None = None) -> Tuple[np.ndarray, int, List[float]]:
    """CG preconditioned by the additive MG method; (x, iterations, ||r_k||)."""
    return pcg(h.fine.A, b, lambda r: additive_precond(h, r, nu, omega), x0=x0, tol=tol, maxit=maxit)


def vcycle_pcg(h: Hierarchy, b: np.ndarray, tol: float = 1e-8, maxit: int = 1000, nu_pre: int = 1,
               nu_post: int = 1, omega: float = 2.0 / 3.0,
               x0: np.ndarray | None = None) -> Tuple[np.ndarray, int, List[float]]:
    """CG preconditioned by one V-cycle; (x, iterations, ||r_k||)."""
    return pcg(h.fine.A, b, lambda r: vcycle(h, r, nu_pre, nu_post, omega), x0=x0, tol=tol, maxit=maxit)
