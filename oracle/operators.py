"""Operators of the oracle: FD matrix, transfers, Galerkin product (FP64).

Sec. 1 (eq. (1)) poses -div(K grad u) = f with Dirichlet data; the paper
discretises with FEM.  The workloads here use the 5-/7-point finite-difference
form on the unit square/cube with homogeneous Dirichlet boundary, mesh width
h = 1/(n+1), and (for heterogeneous kappa) harmonic-mean face coefficients.

Sec. 2.1 defines prolongations P (coarse -> fine) between nested spaces and
restrictions as their transpose.  Here P is tensor-product linear
interpolation, R = 2^{-d} P^T (full weighting; the power-of-two scale changes
no direction, see DESIGN), and coarse operators are the Galerkin products
R A P built by sparse matrix products.

Index order everywhere: x fastest, i.e. flat = i + n*(j + n*k).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _face_coeffs_1axis(kappa: np.ndarray, axis: int) -> np.ndarray:
    """Harmonic means 2 ka kb / (ka + kb) between neighbours along ``axis``.

    ``kappa`` lives on the (n+2)^d node grid including boundary nodes.  The
    result has one entry per face, i.e. (n+1) along ``axis``.
    """
    a = np.take(kappa, np.arange(kappa.shape[axis] - 1), axis=axis)
    b = np.take(kappa, np.arange(1, kappa.shape[axis]), axis=axis)
    return 2.0 * a * b / (a + b)


def fd_matrix(dim: int, n: int, kappa: np.ndarray | None = None) -> sp.csr_matrix:
    """The FD matrix of -div(kappa grad u), Dirichlet u=0, h = 1/(n+1).

    Row i:  A_ii = h^-2 sum_f kappa_f over the 2d faces of node i,
            A_ij = -h^-2 kappa_f for each interior neighbour j across face f.
    With kappa = None every kappa_f = 1 (the 5-/7-point Laplacian).
    Built face by face with explicit index arithmetic, then summed.
    """
    N = n ** dim
    h2inv = float((n + 1) ** 2)
    idx = np.arange(N).reshape((n,) * dim)  # indexed [k, j, i] (x last = fastest)
    rows, cols, vals = [], [], []
    diag = np.zeros((n,) * dim)
    for d_ax in range(dim):
        ax = dim - 1 - d_ax  # numpy axis of spatial direction d_ax (x is last)
        if kappa is None:
            kf = np.ones(tuple(n + 1 if a == ax else n for a in range(dim)))
        else:
            # faces along ax between node planes 0..n+1 (incl. boundary), for
            # interior positions in the other axes
            inner = tuple(slice(1, n + 1) if a != ax else slice(None) for a in range(dim))
            kf = _face_coeffs_1axis(kappa[inner], ax)
        # face f between plane f and plane f+1 (node-grid planes, 0 = boundary)
        lo = np.take(kf, np.arange(0, n), axis=ax)      # face on the low side of interior plane p (=f p)
        hi = np.take(kf, np.arange(1, n + 1), axis=ax)  # face on the high side
        diag += lo + hi
        # off-diagonal couplings between interior planes p and p+1 (face p+1)
        a_idx = np.take(idx, np.arange(0, n - 1), axis=ax).ravel()
        b_idx = np.take(idx, np.arange(1, n), axis=ax).ravel()
        w = np.take(kf, np.arange(1, n), axis=ax).ravel()
        rows += [a_idx, b_idx]
        cols += [b_idx, a_idx]
        vals += [-w, -w]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals) * h2inv,
                       (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()


def interp_1d(n: int) -> sp.csr_matrix:
    """1-D linear interpolation from nc = floor(n/2) coarse to n fine nodes.

    Fine nodes are 1..n (0 and n+1 are the Dirichlet boundary); coarse node I
    (1..nc) sits on fine node 2I.  A fine node on a coarse node takes weight 1;
    a fine node between two coarse nodes takes 1/2 from each, a boundary
    neighbour contributing 0.  Returned 0-based, shape (n, nc).
    """
    nc = n // 2
    rows, cols, vals = [], [], []
    for I in range(1, nc + 1):
        f = 2 * I
        for fi, w in ((f - 1, 0.5), (f, 1.0), (f + 1, 0.5)):
            if 1 <= fi <= n:
                rows.append(fi - 1)
                cols.append(I - 1)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def prolongation(dim: int, n: int) -> sp.csr_matrix:
    """Tensor-product interpolation P = p (x) ... (x) p, fine n^d <- coarse nc^d.

    With x fastest, the Kronecker factor of the slowest axis comes first.
    """
    p = interp_1d(n)
    P = p
    for _ in range(dim - 1):
        P = sp.kron(p, P, format="csr")
    return P.tocsr()


def restriction(dim: int, n: int) -> sp.csr_matrix:
    """Full weighting R = 2^{-d} P^T (transpose of interpolation, Sec. 2.1)."""
    return (prolongation(dim, n).T * (0.5 ** dim)).tocsr()


def symmetrise_upper(A: sp.spmatrix) -> sp.csr_matrix:
    """Keep the upper triangle (incl. diagonal) of A and mirror it."""
    U = sp.triu(A, k=0, format="csr")
    S = U + sp.triu(A, k=1, format="csr").T
    return S.tocsr()


def galerkin(A: sp.spmatrix, P: sp.spmatrix, R: sp.spmatrix) -> sp.csr_matrix:
    """Coarse operator R A P, stored symmetrised (upper triangle mirrored)."""
    Ac = (R @ (A @ P)).tocsr()
    Ac.sum_duplicates()
    return symmetrise_upper(Ac)
