"""Closed-form pins for the oracle's preconditioned CG (oracle/pcg.py).

Facts of the method (exact arithmetic, to rounding here):
  * CG on an SPD matrix with k distinct eigenvalues reaches the solution in
    at most k iterations (the Krylov space then contains A^{-1} b);
  * PCG with the exact inverse as preconditioner converges in one
    iteration, and with a preconditioner M the iterates are those of CG on
    the symmetrically preconditioned system;
  * the residuals are mutually M^{-1}-orthogonal (r_i . z_j = 0 for i != j)
    and the directions mutually A-conjugate (p_i . A p_j = 0).
A plausible slip (a wrong sign in the x or r update, beta taken as
rz_old / rz_new, alpha from r.r instead of r.z) breaks at least one pin.
"""
import numpy as np

from oracle.pcg import pcg


def spd_with_spectrum(eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((len(eigs), len(eigs))))
    return (Q * np.asarray(eigs, dtype=float)) @ Q.T


def test_three_distinct_eigenvalues_three_iterations():
    eigs = [1.0] * 10 + [5.0] * 12 + [40.0] * 8
    A = spd_with_spectrum(eigs, 1)
    b = np.random.default_rng(2).standard_normal(len(eigs))
    x, k, hist = pcg(A, b, lambda r: r, tol=1e-13, maxit=50)
    assert k <= 3
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    x2, k2, _ = pcg(A, b, lambda r: r, tol=1e-13, maxit=2)
    assert k2 == 2 and np.linalg.norm(A @ x2 - b) > 1e-6 * np.linalg.norm(b)   # not yet after two


def test_exact_inverse_preconditioner_one_iteration():
    A = spd_with_spectrum(np.linspace(1.0, 1e3, 40), 3)
    b = np.random.default_rng(4).standard_normal(40)
    Ainv = np.linalg.inv(A)
    x, k, _ = pcg(A, b, lambda r: Ainv @ r, tol=1e-12)
    assert k == 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_matches_cg_on_the_split_preconditioned_system():
    """PCG with M = L L^T equals CG on L^-1 A L^-T, mapped back, iterate by iterate."""
    A = spd_with_spectrum(np.geomspace(1.0, 1e4, 30), 5)
    b = np.random.default_rng(6).standard_normal(30)
    d = np.abs(np.diag(A)) + 1.0
    L = np.diag(np.sqrt(d))           # M = diag(d): preconditioner r -> r / d
    Li = np.diag(1.0 / np.sqrt(d))
    for k in (1, 3, 7):
        x, it, _ = pcg(A, b, lambda r: r / d, tol=0.0, maxit=k)
        y, it2, _ = pcg(Li @ A @ Li, Li @ b, lambda r: r, tol=0.0, maxit=k)
        assert it == it2 == k
        assert np.linalg.norm(x - Li @ y) <= 1e-10 * np.linalg.norm(x)


def test_orthogonality_and_conjugacy():
    """Residuals M^-1-orthogonal and directions A-conjugate over the first
    iterations (recovered from consecutive iterates: p_k ~ x_{k+1} - x_k)."""
    A = spd_with_spectrum(np.linspace(1.0, 50.0, 25), 7)
    b = np.random.default_rng(8).standard_normal(25)
    d = 1.0 + np.arange(25) / 25.0
    xs = [np.zeros(25)]
    for k in range(1, 7):
        xs.append(pcg(A, b, lambda r: r / d, tol=0.0, maxit=k)[0])
    rs = [b - A @ x for x in xs]
    zs = [r / d for r in rs]
    ps = [xs[k + 1] - xs[k] for k in range(6)]
    for i in range(6):
        for j in range(i):
            assert abs(rs[i] @ zs[j]) <= 1e-9 * np.linalg.norm(rs[i]) * np.linalg.norm(zs[j])
            assert abs(ps[i] @ A @ ps[j]) <= 1e-9 * np.sqrt((ps[i] @ A @ ps[i]) * (ps[j] @ A @ ps[j]))


def test_zero_rhs_and_exact_start():
    A = spd_with_spectrum([1.0, 2.0, 3.0], 9)
    x, k, hist = pcg(A, np.zeros(3), lambda r: r)
    assert k == 0 and np.all(x == 0.0)
    b = np.array([1.0, -2.0, 0.5])
    xs = np.linalg.solve(A, b)
    x, k, _ = pcg(A, b, lambda r: r, x0=xs, tol=1e-8)
    assert k == 0
