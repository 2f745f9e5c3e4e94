"""Pins for the A-orthogonalisation of the next block against the stored
window (Sec. 2.2, the truncated sum over j) in its classical form (every
beta_j from Z) and the modified Gram-Schmidt variant.

Facts used:
  * one stored block: both forms are Z - P_1 G_1^+ Q_1^T Z, A-orthogonal to
    P_1 (closed form);
  * stored blocks that are mutually A-orthogonal: the two forms agree and
    the result is A-orthogonal to every block;
  * stored blocks that are not: the modified form takes the last block's
    projection last, so its result is A-orthogonal to that block; the
    classical form's in general is not (this tells the forms apart);
  * in MPCG every block was made A-orthogonal to the m blocks before it, so
    the blocks of a window are mutually A-orthogonal and the two forms give
    the same iterates up to rounding (m = 5).
"""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy, mpcg

RNG = np.random.default_rng(1234)


def spd(n):
    M = RNG.standard_normal((n, n))
    return M @ M.T + n * np.eye(n)


def stored(A, P):
    Q = A @ P
    return (P, Q, np.linalg.inv(P.T @ Q))


def rel_aorth(A, P, X):
    return np.abs(P.T @ A @ X).max() / (np.linalg.norm(A @ P) * np.linalg.norm(X))


def test_single_block_closed_form():
    A = spd(30)
    P1 = RNG.standard_normal((30, 3))
    Z = RNG.standard_normal((30, 4))
    w = [stored(A, P1)]
    expect = Z - P1 @ np.linalg.solve(P1.T @ A @ P1, P1.T @ A @ Z)
    for orth in ("cgs", "mgs"):
        Pn = mpcg.a_orthogonalize(Z, w, orth)
        assert np.abs(Pn - expect).max() <= 1e-12 * np.abs(expect).max()
        assert rel_aorth(A, P1, Pn) <= 1e-13


def test_mutually_orthogonal_blocks_agree():
    A = spd(30)
    V = RNG.standard_normal((30, 6))
    R = np.linalg.cholesky(V.T @ A @ V).T           # V^T A V = R^T R
    Wm = V @ np.linalg.inv(R)                       # W^T A W = I
    w = [stored(A, Wm[:, 2 * j:2 * j + 2]) for j in range(3)]
    Z = RNG.standard_normal((30, 4))
    c = mpcg.a_orthogonalize(Z, w, "cgs")
    m = mpcg.a_orthogonalize(Z, w, "mgs")
    assert np.abs(c - m).max() <= 1e-12 * np.abs(c).max()
    for (Pj, _, _) in w:
        assert rel_aorth(A, Pj, c) <= 1e-13 and rel_aorth(A, Pj, m) <= 1e-13


def test_non_orthogonal_blocks_tell_the_forms_apart():
    A = spd(30)
    w = [stored(A, RNG.standard_normal((30, 2))) for _ in range(2)]
    Z = RNG.standard_normal((30, 3))
    c = mpcg.a_orthogonalize(Z, w, "cgs")
    m = mpcg.a_orthogonalize(Z, w, "mgs")
    last = w[-1][0]
    assert rel_aorth(A, last, m) <= 1e-13
    assert rel_aorth(A, last, c) > 1e-3
    with pytest.raises(ValueError):
        mpcg.a_orthogonalize(Z, w, "householder")


def test_window_solves_agree_in_both_forms():
    prob = W.GridProblem("t", 2, 31, 4, 5, kappa_seed=5)
    h = hierarchy.build(2, 31, 4, kappa=W.kappa_field(prob))
    b = W.rhs(31 * 31, 5)
    for m in (1, 5):
        c = mpcg.mpcg(h, b, tol=1e-8, maxit=500, m=m, orth="cgs")
        g = mpcg.mpcg(h, b, tol=1e-8, maxit=500, m=m, orth="mgs")
        assert c.status == g.status == mpcg.OK
        assert abs(c.iterations - g.iterations) <= 1
        if m == 1:
            assert np.array_equal(c.x, g.x)
        k = min(c.iterations, g.iterations, 15)
        ck = mpcg.mpcg(h, b, tol=0.0, maxit=k, m=m, orth="cgs").x
        gk = mpcg.mpcg(h, b, tol=0.0, maxit=k, m=m, orth="mgs").x
        assert np.linalg.norm(ck - gk) <= 1e-8 * np.linalg.norm(ck), m
