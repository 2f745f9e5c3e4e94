"""Additive-MG multipreconditioned CG, Algorithm 1 of Sec. 2.2 (FP64 oracle).

Each iteration takes the L+1 additive-MG level corrections
z^l = P_l^L S_l^nu (R_L^l r) (Sec. 2.2, the block P_k, columns ordered
coarsest -> finest) as separate search directions, combines them with the
energy-minimising coefficients alpha = (P^T A P)^+ (P^T r), eq. (4), and
A-orthogonalises the next block against the last m stored blocks.

Readings where the paper is silent or ambiguous (all listed in DESIGN):
  * smoother start c_0 = 0, same nu sweeps on every level (eq. (2), (3));
  * (P^T A P)^{-1} may be singular (Sec. 2.2); a pseudo-inverse from the
    eigen-decomposition of the Jacobi-scaled Gram is used, dropping
    eigenvalues <= tau (default 64 * b * 2^-53);
  * the same G_k^+ serves alpha_k and the beta of the next orthogonalisation;
  * A P_{k+1} is recomputed from P_{k+1} (not updated by recurrence);
  * convergence: ||r_k||_2 <= tol ||b||_2 on the recursively updated r,
    tested after every update; iterations = number of x updates;
  * the truncation sum over j runs over the last m stored blocks (m = 1 is
    the "previous block only" form), in classical Gram-Schmidt form (every
    beta_j from Z_{k+1}); modified Gram-Schmidt is the variant ``orth="mgs"``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .hierarchy import Hierarchy, prolong_from, restrict_to
from .smoother import jacobi

OK, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, -4


def default_tau(b: int, unit_roundoff: float = 2.0 ** -53) -> float:
    return 64.0 * b * unit_roundoff


def level_correction(h: Hierarchy, r: np.ndarray, l: int, nu: int, omega: float,
                     coarse_exact: bool = False) -> np.ndarray:
    """z^l = P_l^L S_l^nu (R_L^l r)  (Algorithm 1, "corrections from all levels")."""
    g = restrict_to(h, r, l)
    lev = h.levels[l]
    if l == 0 and coarse_exact:
        c = np.linalg.solve(lev.A.toarray(), g)
    else:
        c = jacobi(lev.A, lev.D, g, nu, omega)
    return prolong_from(h, c, l)


def mg_block(h: Hierarchy, r: np.ndarray, nu: int = 2, omega: float = 2.0 / 3.0,
             coarse_exact: bool = False) -> np.ndarray:
    """Z = [z^0 | z^1 | ... | z^L], n x (L+1), coarsest column first."""
    cols = [level_correction(h, r, l, nu, omega, coarse_exact) for l in range(h.L + 1)]
    return np.stack(cols, axis=1)


@dataclass
class Pinv:
    """Pseudo-inverse of a symmetric PSD b x b Gram matrix and its rank."""
    Gplus: np.ndarray
    rank: int


def pinv_gram(G: np.ndarray, tau: float) -> Pinv:
    """Jacobi-scaled eigen pseudo-inverse.

    Columns with a positive finite diagonal are active.  With S =
    diag(G_ii^{-1/2}) on them, Ghat = S G S has unit diagonal; its
    eigenpairs (library ``eigh``) with lambda > tau are kept and
    G^+ = S V Lambda^+ V^T S (zero rows/columns for inactive directions).
    """
    b = G.shape[0]
    d = np.diag(G)
    active = np.isfinite(d) & (d > 0.0)
    Gplus = np.zeros((b, b))
    if not np.any(active):
        return Pinv(Gplus, 0)
    ia = np.nonzero(active)[0]
    s = 1.0 / np.sqrt(d[ia])
    Ga = G[np.ix_(ia, ia)]
    if not np.all(np.isfinite(Ga)):
        return Pinv(Gplus, 0)
    Ghat = (Ga * s[:, None]) * s[None, :]
    lam, V = np.linalg.eigh(Ghat)
    keep = lam > tau
    Vk = V[:, keep]
    inner = (Vk / lam[keep][None, :]) @ Vk.T
    Gplus[np.ix_(ia, ia)] = (inner * s[:, None]) * s[None, :]
    return Pinv(Gplus, int(np.count_nonzero(keep)))


def gram(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """P^T Q computed as its upper triangle and mirrored (symmetric Gram)."""
    b = P.shape[1]
    G = np.zeros((b, b))
    for i in range(b):
        for j in range(i, b):
            G[i, j] = P[:, i] @ Q[:, j]
            G[j, i] = G[i, j]
    return G


@dataclass
class Result:
    x: np.ndarray
    iterations: int
    status: int
    resnorms: List[float]                 # ||r_k||_2 for k = 0..iterations
    alphas: List[np.ndarray] = field(default_factory=list)
    ranks: List[int] = field(default_factory=list)
    snapshots: Dict[int, np.ndarray] = field(default_factory=dict)
    bnorm: float = 0.0


def a_orthogonalize(Z: np.ndarray, window, orth: str = "cgs") -> np.ndarray:
    """The next block P_{k+1} from Z_{k+1} and the stored (P_j, Q_j = A P_j,
    G_j^+) of the window, oldest first (Sec. 2.2, the truncated sum over j):
    P_{k+1} = Z - sum_j P_j beta_j with beta_j = G_j^+ Q_j^T V, where V is
    Z for every j (classical Gram-Schmidt, ``"cgs"``) or the block as far as
    it is orthogonalised, block after block (modified, ``"mgs"``).  The two
    agree in exact arithmetic when the stored blocks are mutually
    A-orthogonal, as the window's blocks are."""
    if orth not in ("cgs", "mgs"):
        raise ValueError("orth must be 'cgs' or 'mgs'")
    Pn = Z.copy()
    for (Pj, Qj, Gpj) in window:
        beta = Gpj @ (Qj.T @ (Z if orth == "cgs" else Pn))
        Pn = Pn - Pj @ beta
    return Pn


def mpcg(h: Hierarchy, b: np.ndarray, x0: Optional[np.ndarray] = None,
         tol: float = 1e-8, maxit: int = 1000, m: int = 1, nu: int = 2,
         omega: float = 2.0 / 3.0, tau: Optional[float] = None,
         extra: Optional[Callable[[np.ndarray], np.ndarray]] = None,
         coarse_exact: bool = False, snapshots: Sequence[int] = (),
         callback: Optional[Callable[[int, np.ndarray, np.ndarray], None]] = None,
         orth: str = "cgs") -> Result:
    """Algorithm 1 with truncation window m.

    ``extra``, if given, maps r to one more search direction appended after
    the level corrections (a non-finite direction is replaced by zero, so
    the energy minimisation simply gets a zero column).
    ``callback(k, x_k, P_k)`` is called with each iterate and the block used
    from it (tests of conjugacy and monotone energy use it).
    """
    A = h.fine.A
    n = A.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    nb = float(np.linalg.norm(b))
    A_ = A

    def directions(r):
        Z = mg_block(h, r, nu, omega, coarse_exact)
        if extra is not None:
            d = np.asarray(extra(r), dtype=np.float64)
            if not np.all(np.isfinite(d)):
                d = np.zeros(n)
            Z = np.concatenate([Z, d[:, None]], axis=1)
        return Z

    res = Result(x, 0, OK, [], bnorm=nb)
    if nb == 0.0:
        res.x = np.zeros(n)
        res.resnorms = [0.0]
        return res
    r = b - A_ @ x                                    # r_0 = b - A x_0
    rn = float(np.linalg.norm(r))
    res.resnorms.append(rn)
    if 0 in snapshots:
        res.snapshots[0] = x.copy()
    if not np.isfinite(rn):
        res.status = NONFINITE
        return res
    if rn <= tol * nb:
        return res
    Z = directions(r)                                 # P_0 = Z_0 = MG(r_0)
    bw = Z.shape[1]
    if tau is None:
        tau = default_tau(bw)
    P = Z
    Q = np.column_stack([A_ @ P[:, j] for j in range(bw)])
    G = gram(P, Q)
    pv = pinv_gram(G, tau)
    window = []                                       # stored (P_j, Q_j, G_j^+)
    k = 0
    while True:
        if pv.rank == 0:
            res.status = BREAKDOWN
            break
        g = P.T @ r
        alpha = pv.Gplus @ g                          # alpha_k = (P^T A P)^+ P^T r
        res.alphas.append(alpha.copy())
        res.ranks.append(pv.rank)
        if callback is not None:
            callback(k, x.copy(), P.copy())
        x = x + P @ alpha                             # x_{k+1}
        r = r - Q @ alpha                             # r_{k+1}
        k += 1
        rn = float(np.linalg.norm(r))
        res.resnorms.append(rn)
        if k in snapshots:
            res.snapshots[k] = x.copy()
        if not np.isfinite(rn):
            res.status = NONFINITE
            break
        if rn <= tol * nb:
            break
        if k >= maxit:
            res.status = MAXIT
            break
        window.append((P, Q, pv.Gplus))
        if len(window) > m:
            window.pop(0)
        Z = directions(r)                             # Z_{k+1} = MG(r_{k+1})
        P = a_orthogonalize(Z, window, orth)          # P_{k+1}, A-orthogonal to the window
        Q = np.column_stack([A_ @ P[:, j] for j in range(bw)])
        G = gram(P, Q)
        pv = pinv_gram(G, tau)
    res.x = x
    res.iterations = k
    return res
