"""Pins for the oracle's operators, transfers, Galerkin levels and smoother.

Each check compares the oracle with something fixed independently of it:
closed-form eigenpairs of the discrete Laplacian, hat functions sampled by
scalar loops, hand-derived Galerkin stencils (tests/golden), the closed form
of damped Jacobi on an eigenvector, and dense brute force.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import hierarchy, operators as ops, smoother
from oracle.mpcg import level_correction

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sine_mode(dim, n, ks):
    h = 1.0 / (n + 1)
    v = None
    for ax in range(dim):  # ks[0] along x (fastest)
        s = np.sin(ks[ax] * math.pi * h * np.arange(1, n + 1))
        v = s if v is None else np.multiply.outer(s, v)
    return v.reshape(-1)


def laplace_eig(dim, n, ks):
    h = 1.0 / (n + 1)
    return 4.0 / h ** 2 * sum(math.sin(k * math.pi * h / 2) ** 2 for k in ks)


@pytest.mark.parametrize("dim,n,ks", [(2, 7, (1, 1)), (2, 7, (3, 5)), (2, 8, (2, 7)),
                                      (3, 5, (1, 2, 3)), (3, 6, (4, 1, 2))])
def test_fd_sine_eigenpairs(dim, n, ks):
    A = ops.fd_matrix(dim, n)
    v = sine_mode(dim, n, ks)
    lam = laplace_eig(dim, n, ks)
    np.testing.assert_allclose(A @ v, lam * v, rtol=0, atol=1e-10 * lam)


def test_fd_symmetric_rowsums():
    for dim, n in ((2, 9), (3, 5)):
        A = ops.fd_matrix(dim, n)
        assert abs(A - A.T).max() == 0.0
        Ad = A.toarray()
        grid = np.arange(n ** dim).reshape((n,) * dim)
        inner = grid[(slice(1, n - 1),) * dim].ravel()
        assert np.all(Ad[inner].sum(axis=1) == 0.0)


def test_fd_kappa_one_is_poisson_bitwise():
    for dim, n in ((2, 9), (3, 6)):
        A0 = ops.fd_matrix(dim, n)
        A1 = ops.fd_matrix(dim, n, np.ones((n + 2,) * dim))
        assert (A0 != A1).nnz == 0


def test_fd_heterogeneous_entries_by_hand():
    dim, n = 3, 5
    rng = np.random.default_rng(11)
    kap = np.exp(rng.standard_normal((n + 2,) * 3))
    A = ops.fd_matrix(dim, n, kap).toarray()
    h2 = (n + 1) ** 2

    def hm(a, b):
        return 2 * a * b / (a + b)
    for (i, j, k) in [(0, 0, 0), (2, 3, 1), (4, 4, 4), (1, 0, 3)]:
        row = i + n * (j + n * k)
        K = lambda a, b, c: kap[c + 1, b + 1, a + 1]  # node-grid value at interior (a,b,c)
        faces = []
        for d, (di, dj, dk) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            for s in (-1, 1):
                a, b, c = i + s * di, j + s * dj, k + s * dk
                kf = hm(K(i, j, k), K(a, b, c))
                faces.append(kf)
                if 0 <= a < n and 0 <= b < n and 0 <= c < n:
                    col = a + n * (b + n * c)
                    assert A[row, col] == pytest.approx(-h2 * kf, rel=1e-14)
        assert A[row, row] == pytest.approx(h2 * sum(faces), rel=1e-14)


@pytest.mark.parametrize("n", [7, 8, 15, 31])
def test_interp_is_hat_function(n):
    p = ops.interp_1d(n).toarray()
    h = 1.0 / (n + 1)
    nc = n // 2
    for f in range(1, n + 1):
        for I in range(1, nc + 1):
            hat = max(0.0, 1.0 - abs(f - 2 * I) / 2.0)  # hat of width 2h at node 2I
            assert p[f - 1, I - 1] == hat


def test_tensor_prolongation_weights():
    # weights 1, 1/2, 1/4, 1/8 of trilinear interpolation around coarse node (2,1,3)
    n = 9
    P = ops.prolongation(3, n).toarray()
    nc = n // 2
    I, J, K = 2, 1, 3  # 1-based coarse, at fine (4, 2, 6)
    col = (I - 1) + nc * ((J - 1) + nc * (K - 1))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                f = (2 * I + dx - 1) + n * ((2 * J + dy - 1) + n * (2 * K + dz - 1))
                expect = 0.5 ** (abs(dx) + abs(dy) + abs(dz))
                assert P[f, col] == expect
    assert P[:, col].sum() == 8.0


def test_full_weighting_adjoint_and_constants():
    rng = np.random.default_rng(5)
    for dim, n in ((2, 15), (3, 7)):
        P = ops.prolongation(dim, n)
        R = ops.restriction(dim, n)
        u = rng.standard_normal(P.shape[0])
        v = rng.standard_normal(P.shape[1])
        assert (R @ u) @ v == pytest.approx(0.5 ** dim * (u @ (P @ v)), rel=1e-13)
        # n odd: every coarse node has all its fine neighbours, FW of 1 is 1
        np.testing.assert_array_equal(R @ np.ones(P.shape[0]), np.ones(P.shape[1]))


def _stencil_at(A, dim, n, center):
    """Dense stencil of row ``center`` (tuple of 0-based coords, x first)."""
    Ad = A.toarray()
    row = sum(c * n ** a for a, c in enumerate(center))
    st = np.zeros((3,) * dim)
    for off in np.ndindex(*(3,) * dim):
        nb = [center[a] + off[dim - 1 - a] - 1 for a in range(dim)]
        col = sum(c * n ** a for a, c in enumerate(nb))
        st[off] = Ad[row, col]
    return st


def _closed_form_stencil(dim, level_from_fine, H):
    """Galerkin stencil from the hand-derived 1-D factors in tests/golden."""
    with open(os.path.join(GOLDEN, "galerkin_1d_factors.json")) as f:
        g = json.load(f)
    M = np.array([float(Fraction(s)) for s in g["mass"][str(level_from_fine)]])
    T = np.array([-1.0, 2.0, -1.0]) / H ** 2
    st = np.zeros((3,) * dim)
    for ax in range(dim):
        fac = [M] * dim
        fac[ax] = T
        t = fac[0]
        for f in fac[1:]:
            t = np.multiply.outer(t, f)
        st += t
    return st


@pytest.mark.parametrize("dim,n", [(2, 31), (3, 15)])
def test_galerkin_interior_stencils_closed_form(dim, n):
    h = hierarchy.build(dim, n, 3)
    for depth in (1, 2):
        lev = h.levels[h.L - depth]
        nl = lev.n
        H = (2 ** depth) / (n + 1)
        c = nl // 2
        got = _stencil_at(lev.A, dim, nl, (c,) * dim)
        expect = _closed_form_stencil(dim, depth, H)
        np.testing.assert_allclose(got, expect, rtol=1e-13, atol=1e-12 * abs(expect).max())


def test_galerkin_appendix_values_2d_level1():
    # 2D level 1: H^-2 [-1/4 -1/2 -1/4; -1/2 3 -1/2; -1/4 -1/2 -1/4]
    n = 15
    h = hierarchy.build(2, n, 2)
    lev = h.levels[0]
    H = 2.0 / (n + 1)
    got = _stencil_at(lev.A, 2, lev.n, (3, 3)) * H ** 2
    np.testing.assert_allclose(got, [[-.25, -.5, -.25], [-.5, 3, -.5], [-.25, -.5, -.25]], atol=1e-13)


def test_galerkin_levels_spd_symmetric():
    prob = W.GridProblem("t", 3, 15, 3, 0, kappa_seed=7)
    h = hierarchy.build(3, 15, 3, kappa=W.kappa_field(prob))
    for lev in h.levels:
        Ad = lev.A.toarray()
        assert np.array_equal(Ad, Ad.T)
        assert np.linalg.eigvalsh(Ad).min() > 0


def test_jacobi_closed_form_on_eigenvector():
    for dim, n, ks in ((2, 15, (2, 3)), (3, 7, (1, 4, 2))):
        A = ops.fd_matrix(dim, n)
        D = A.diagonal()
        v = sine_mode(dim, n, ks)
        lam = laplace_eig(dim, n, ks)
        d0 = 2 * dim * (n + 1) ** 2
        for nu in (1, 2, 3):
            for omega in (2.0 / 3.0, 0.8):
                c = smoother.jacobi(A, D, v, nu, omega)
                expect = (1 - (1 - omega * lam / d0) ** nu) / lam * v
                np.testing.assert_allclose(c, expect, rtol=0, atol=1e-13 * abs(expect).max())


def _dense_interp_1d(n):
    nc = n // 2
    h = 1.0 / (n + 1)
    return np.array([[max(0.0, 1 - abs(f - 2 * I) / 2.0) for I in range(1, nc + 1)]
                     for f in range(1, n + 1)])


def test_level_correction_dense_brute_force():
    """z^l = P_l^L S_l^nu R_L^l r against dense matrices built independently."""
    dim, n, nl = 2, 15, 3
    nu, omega = 2, 2.0 / 3.0
    rng = np.random.default_rng(3)
    Afine = ops.fd_matrix(dim, n).toarray()
    h = hierarchy.build(dim, n, nl)
    sizes = [15, 7, 3]
    Ps = []
    for s in sizes[:-1]:
        p = _dense_interp_1d(s)
        Ps.append(np.kron(p, p))     # fine(s) <- coarse
    As = [Afine]
    for P in Ps:
        As.append(0.25 * P.T @ As[-1] @ P)
    r = rng.standard_normal(n * n)
    for depth in range(nl):          # depth 0 = finest
        Pc = np.eye(n * n)
        for P in Ps[:depth]:
            Pc = Pc @ P
        Al = As[depth]
        Dinv = np.diag(1.0 / np.diag(Al))
        E = np.eye(Al.shape[0]) - omega * Dinv @ Al
        S = sum(np.linalg.matrix_power(E, i) for i in range(nu)) @ (omega * Dinv)
        Rc = (0.25 ** depth) * Pc.T
        z_expect = Pc @ S @ Rc @ r
        z = level_correction(h, r, h.L - depth, nu, omega)
        np.testing.assert_allclose(z, z_expect, rtol=0, atol=1e-12 * abs(z_expect).max())


def test_level_smoother_spd_for_omega_two_thirds():
    """omega * lambda_max(D^-1 A_l) < 2 on every level, so S_l^nu is SPD."""
    prob = W.GridProblem("t", 3, 15, 3, 0, kappa_seed=3)
    for kap in (None, W.kappa_field(prob)):
        h = hierarchy.build(3, 15, 3, kappa=kap)
        for lev in h.levels:
            Ad = lev.A.toarray()
            Dm = np.diag(1 / np.sqrt(lev.D))
            lmax = np.linalg.eigvalsh(Dm @ Ad @ Dm).max()
            assert (2.0 / 3.0) * lmax < 2.0


def test_not_spd_rejected():
    A = ops.fd_matrix(2, 7).tolil()
    A[5, 5] = -1.0
    with pytest.raises(hierarchy.NotSPDError):
        hierarchy.build(2, 7, 2, A=A.tocsr())
