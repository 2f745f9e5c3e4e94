"""Textbook preconditioned CG (FP64), used only as a pin for MPCG.

With a single level (the block has one column z = S^nu r) MPCG is, in exact
arithmetic, PCG with the preconditioner S^nu; this routine is the classical
two-term recurrence (Hestenes-Stiefel form), written independently of mpcg.
It is also the additive-MG-PCG comparator of Sec. 3 when ``precond`` is the
summed additive correction of eq. (3).
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np


def pcg(A, b: np.ndarray, precond: Callable[[np.ndarray], np.ndarray],
        x0: np.ndarray | None = None, tol: float = 1e-8,
        maxit: int = 1000) -> Tuple[np.ndarray, int, List[float]]:
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    hist = [float(np.linalg.norm(r))]
    if hist[0] <= tol * nb:
        return x, 0, hist
    z = precond(r)
    p = z.copy()
    rz = r @ z
    k = 0
    while k < maxit:
        Ap = A @ p
        a = rz / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        k += 1
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= tol * nb:
            break
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, k, hist
