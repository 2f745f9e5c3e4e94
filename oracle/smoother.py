"""Damped-Jacobi smoothing S_l^nu of eq. (2) (FP64 oracle).

Eq. (2) writes nu steps of a stationary iteration with preconditioner M_l
from a start c_0.  Here M_l = omega^{-1} D_l (damped Jacobi) and c_0 = 0, so
S_l^nu is a fixed linear operator:

    c_{s+1} = c_s + omega * ((g - A_l c_s) / D_l),   s = 0..nu-1.

The division form omega * (res / D) is the one used on both sides.  The same
nu sweeps are applied on every level, the coarsest included (S_0 is the
paper's unspecified "approximate inverse").
"""
from __future__ import annotations

import numpy as np


def jacobi(A, D: np.ndarray, g: np.ndarray, nu: int, omega: float) -> np.ndarray:
    c = np.zeros_like(g)
    for _ in range(nu):
        c = c + omega * ((g - A @ c) / D)
    return c
