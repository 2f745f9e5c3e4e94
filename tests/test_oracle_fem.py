"""Pins for the bilinear finite elements of Example 1 (Sec. 3) and for the
input stencil the GPU path receives.

Facts used:
  * isotropic K: the textbook bilinear Laplacian stencil [-1 -1 -1; -1 8 -1;
    -1 -1 -1] / 3;
  * the stiffness is linear in (kxx, kyy), and swapping kxx and kyy swaps
    the x and y axes;
  * the assembled matrix is symmetric positive definite;
  * O(h^2) nodal convergence to the smooth solution sin(pi x) sin(pi y) of the
    anisotropic problem;
  * the interior stencil read off the quadrature-assembled matrix equals the
    closed tensor-product form the workloads module hands to the solver;
  * lambda_max(D^-1 A) tends to 3 as kxx -> 0, so damped Jacobi needs
    omega < 2/3 there (the Example 1 runs use omega = 1/2);
  * Sec. 3's observations on alpha in the highly anisotropic case: some
    alpha_l are negative, and in the later iterations the finest level
    carries the largest |alpha_l| while the coarse ones shrink.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import workloads as W
from oracle import fem, hierarchy, mpcg


def test_isotropic_stencil_is_textbook():
    st = fem.stencil(12, 1.0, 1.0)
    expect = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3.0
    assert np.abs(st - expect).max() <= 1e-14


def test_linear_in_the_coefficients_and_axis_swap():
    m = 9
    A = fem.stiffness(m, 0.3, 2.5)
    Ax, Ay = fem.stiffness(m, 1.0, 0.0), fem.stiffness(m, 0.0, 1.0)
    assert abs(A - (0.3 * Ax + 2.5 * Ay)).max() <= 1e-13
    n = m - 1
    perm = np.arange(n * n).reshape(n, n).T.reshape(-1)      # (i, j) -> (j, i)
    B = fem.stiffness(m, 2.5, 0.3)[perm][:, perm]
    assert abs(A - B).max() <= 1e-13


def test_spd():
    A = fem.stiffness(10, 1e-4).toarray()
    assert np.abs(A - A.T).max() <= 1e-15
    assert np.linalg.eigvalsh(A).min() > 0.0


def _nodal_error(m, kxx, kyy):
    n = m - 1
    x = np.arange(1, m) / m
    u = np.outer(np.sin(math.pi * x), np.sin(math.pi * x)).reshape(-1)     # symmetric in x, y
    f = math.pi ** 2 * (kxx + kyy) * u
    # consistent load of the bilinear interpolant of f: M f with the Q1 mass
    m1 = sp.diags([np.full(n - 1, 1.0), np.full(n, 4.0), np.full(n - 1, 1.0)], [-1, 0, 1]) / 6.0 / m
    M = sp.kron(m1, m1)
    A = fem.stiffness(m, kxx, kyy)
    uh = sla.spsolve(A.tocsc(), M @ f)
    return np.abs(uh - u).max()


def test_second_order_convergence():
    for kxx in (1.0, 0.05):
        e1, e2 = _nodal_error(16, kxx, 1.0), _nodal_error(32, kxx, 1.0)
        assert 3.5 < e1 / e2 < 4.5, (kxx, e1, e2)


def test_workload_stencil_matches_assembly():
    for kxx in (1.0, 1e-1, 1e-4, 1e-7, 3.0):
        assert np.abs(W.example1_stencil(kxx) - fem.stencil(20, kxx)).max() <= 1e-14
    b = W.example1_rhs(20)
    assert b.size == 19 * 19 and np.allclose(b, fem.load(20))


def test_jacobi_spectrum_tends_to_three():
    lams = []
    for kxx in (1.0, 1e-2, 1e-6):
        A = fem.stiffness(32, kxx)
        d = 1.0 / np.sqrt(A.diagonal())
        lams.append(sla.eigsh(sp.diags(d) @ A @ sp.diags(d), k=1, which="LA")[0][0])
    assert lams[0] < 1.6 and 2.95 < lams[2] < 3.0 and lams[0] < lams[1] < lams[2]


def test_alpha_observations_high_anisotropy():
    m = W.EXAMPLE1_ELEMENTS
    A = fem.stiffness(m, 1e-6)
    h = hierarchy.build(2, m - 1, W.EXAMPLE1_LEVELS, A=A)
    res = mpcg.mpcg(h, fem.load(m), tol=1e-8, m=5, nu=6, omega=0.5, maxit=3000)
    assert res.status == mpcg.OK
    al = np.array(res.alphas)
    assert (al < 0).any()
    late = np.abs(al[-10:])
    assert (late.argmax(axis=1) == al.shape[1] - 1).all()            # finest column largest
    early = np.abs(al[:10])
    assert late[:, :-1].mean() < 0.5 * early[:, :-1].mean()          # coarse levels shrink
