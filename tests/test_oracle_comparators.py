"""Pins for the oracle's comparison methods of Sec. 3 (additive MG-PCG and
MG(V)-PCG).

Facts used:
  * one level, sine eigenvector of the constant-coefficient Laplacian: the
    V-cycle is nu_pre + nu_post damped-Jacobi sweeps from zero, whose
    result is [1 - (1 - omega mu)^nu] / lambda times the eigenvector
    (mu = lambda / D) -- a closed form;
  * the V-cycle equals its error-propagation definition, built from dense
    matrices level by level: E_l = S^post (I - P B_{l-1} R A_l) S^pre,
    B_l = (I - E_l) A_l^{-1}, B_0 = (I - S_0^(pre+post)) A_0^{-1};
  * with nu_pre = nu_post the V-cycle is a symmetric operator and the
    eigenvalues of B A lie in (0, 1] (E is A-self-adjoint with norm < 1);
  * one level: additive MG-PCG is PCG with S^nu, hence MPCG with one level;
  * Sec. 3's ordering on these cases: MG(V)-PCG needs the fewest iterations,
    additive-MG MPCG (m = 5) fewer than additive MG-PCG.
"""
import math

import numpy as np

import workloads as W
from oracle import comparators as C
from oracle import hierarchy, mpcg


def small_problem(dim=2, n=31, nl=4, seed=1, kappa_seed=None):
    prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=kappa_seed)
    h = hierarchy.build(dim, n, nl, kappa=W.kappa_field(prob))
    b = W.rhs(n ** dim, seed)
    return h, b


def test_vcycle_one_level_is_jacobi_closed_form():
    n, omega = 15, 2.0 / 3.0
    hh = 1.0 / (n + 1)
    h = hierarchy.build(2, n, 1)
    x = np.arange(1, n + 1) * hh
    for (p, q, pre, post) in ((1, 1, 1, 1), (3, 5, 2, 2), (7, 2, 1, 2)):
        v = np.outer(np.sin(q * math.pi * x), np.sin(p * math.pi * x)).reshape(-1)   # x fastest
        lam = 4.0 / hh ** 2 * (math.sin(p * math.pi * hh / 2) ** 2 + math.sin(q * math.pi * hh / 2) ** 2)
        mu = lam / (4.0 / hh ** 2)
        expect = (1.0 - (1.0 - omega * mu) ** (pre + post)) / lam * v
        got = C.vcycle(h, v, pre, post, omega)
        assert np.linalg.norm(got - expect) <= 1e-12 * np.linalg.norm(expect)


def _dense_B(h, pre, post, omega):
    """V-cycle operator from its error-propagation definition (dense)."""
    Bs = []
    for l, lev in enumerate(h.levels):
        A = lev.A.toarray()
        Ainv = np.linalg.inv(A)
        I = np.eye(A.shape[0])
        S = I - omega * (A / lev.D[:, None])
        if l == 0:
            E = np.linalg.matrix_power(S, pre + post)
        else:
            P = h.levels[l - 1].P.toarray()
            R = h.levels[l - 1].R.toarray()
            CC = I - P @ Bs[-1] @ R @ A
            E = np.linalg.matrix_power(S, post) @ CC @ np.linalg.matrix_power(S, pre)
        Bs.append((I - E) @ Ainv)
    return Bs[-1]


def test_vcycle_matches_error_propagation_form():
    rng = np.random.default_rng(3)
    for (dim, n, nl, ks, pre, post) in ((2, 15, 3, None, 1, 1), (2, 15, 4, 5, 2, 2), (3, 7, 2, 3, 1, 1),
                                        (2, 13, 3, 2, 3, 1)):
        h, _ = small_problem(dim, n, nl, 1, ks)
        B = _dense_B(h, pre, post, 2.0 / 3.0)
        for _ in range(3):
            r = rng.standard_normal(n ** dim)
            got = C.vcycle(h, r, pre, post)
            assert np.linalg.norm(got - B @ r) <= 1e-11 * np.linalg.norm(B @ r)


def test_vcycle_symmetric_and_spectrum_in_unit_interval():
    rng = np.random.default_rng(4)
    h, _ = small_problem(3, 7, 2, 1, 3)
    u, v = rng.standard_normal(343), rng.standard_normal(343)
    for nu in (1, 2, 3):
        a = u @ C.vcycle(h, v, nu, nu)
        b = v @ C.vcycle(h, u, nu, nu)
        assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)
    h2, _ = small_problem(2, 15, 3, 1, 5)
    B = _dense_B(h2, 1, 1, 2.0 / 3.0)
    lam = np.linalg.eigvals(B @ h2.fine.A.toarray())
    assert np.abs(lam.imag).max() <= 1e-8
    assert lam.real.min() > 0.0 and lam.real.max() <= 1.0 + 1e-10


def test_additive_pcg_one_level_is_one_level_mpcg():
    h, b = small_problem(2, 31, 1, 7)
    for k in (1, 4, 9):
        x_add, _, _ = C.additive_pcg(h, b, tol=0.0, maxit=k)
        res = mpcg.mpcg(h, b, tol=0.0, maxit=k)
        assert np.linalg.norm(x_add - res.x) <= 1e-10 * np.linalg.norm(res.x)


def test_additive_precond_is_symmetric():
    rng = np.random.default_rng(5)
    h, _ = small_problem(3, 15, 3, 1, 3)
    u, v = rng.standard_normal(15 ** 3), rng.standard_normal(15 ** 3)
    a = u @ C.additive_precond(h, v)
    b = v @ C.additive_precond(h, u)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_paper_ordering_of_the_three_methods():
    """Sec. 3: the V-cycle preconditioner is the strongest; additive-MG
    MPCG (m = 5) beats additive MG-PCG.  (On the 2D 45^2 kappa case the
    second claim fails in this setting; DESIGN records it.)"""
    for (dim, n, nl, ks) in ((2, 31, 4, None), (2, 63, 5, None), (3, 15, 3, 3), (3, 31, 4, None), (3, 31, 4, 3)):
        h, b = small_problem(dim, n, nl, 4, ks)
        _, k_add, _ = C.additive_pcg(h, b, 1e-8)
        _, k_v, _ = C.vcycle_pcg(h, b, 1e-8)
        k_mp = mpcg.mpcg(h, b, tol=1e-8, m=5).iterations
        assert k_v < k_mp < k_add, (dim, n, nl, ks, k_v, k_mp, k_add)
