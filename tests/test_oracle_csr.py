"""Pins for the oracle's general hierarchy (given prolongations) and for the
unstructured graph workload fed to the CSR entry point.

Facts used: with the structured prolongations, the general Galerkin
construction gives exactly the structured hierarchy's level operators; the
graph operator is symmetric positive definite and every fine unknown lies
in exactly one aggregate, so the coarse operators stay symmetric positive
definite (P has full column rank); MPCG on it converges and matches a
dense solve on a small instance.
"""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import hierarchy, mpcg


def test_general_hierarchy_matches_structured():
    for (dim, n, nl, ks) in ((2, 31, 4, None), (3, 15, 3, 3)):
        prob = W.GridProblem("t", dim, n, nl, 1, kappa_seed=ks)
        h = hierarchy.build(dim, n, nl, kappa=W.kappa_field(prob))
        Ps = [h.levels[l].P for l in range(nl - 1)]
        g = hierarchy.from_operators(h.fine.A, Ps, 0.5 ** dim)
        for l in range(nl):
            assert abs(h.levels[l].A - g.levels[l].A).max() <= 1e-12 * abs(h.levels[l].A).max()


def test_graph_problem_structure():
    A, Ps, b = W.graph_problem(npts=600, seed=3, nlevels=3)
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0.0
    for P in Ps:
        assert np.all(np.diff(P.indptr) == 1) and np.all(P.data == 1.0)
        assert np.all(np.asarray(P.sum(axis=0)).reshape(-1) >= 1)     # no empty aggregate
    h = hierarchy.from_operators(A, Ps, 1.0)
    for lev in h.levels:
        M = lev.A.toarray()
        assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
        assert np.linalg.eigvalsh(M).min() > 0.0


def test_graph_problem_mpcg_matches_dense_solve():
    A, Ps, b = W.graph_problem(npts=600, seed=3, nlevels=3)
    h = hierarchy.from_operators(A, Ps, 1.0)
    res = mpcg.mpcg(h, b, tol=1e-12, maxit=2000)
    assert res.status == mpcg.OK
    xs = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)
